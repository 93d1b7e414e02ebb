/*
 * pot3d_oracle.c -- FP64 CPU oracle for the potential-field PCG solve.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this code.  The GPU solver library neither
 * links nor calls it, and the two share no source, header or table.
 *
 * What it computes, and where each piece comes from in the paper
 * (Caplan, Mikic & Linker, "From MPI to MPI+OpenACC", arXiv:1709.01126):
 *
 *  - The model (Sec. 2.1): Laplace's equation for the potential, eq. (1), on the
 *    shell R0 <= r <= R1, with
 *      * the surface condition eq. (2) on r = R0, read here with the sign
 *        dPhi/dr = -Br (so B = -grad Phi); the paper's +Br convention gives -Phi;
 *      * the "source surface" condition Phi = 0 on r = R1, or the "closed wall"
 *        Br = 0 on r = R1 (no flux through the top face; the system is then
 *        singular, with the constants as its null space: see orc_rhs_bc and
 *        orc_gauge);
 *      * periodicity in phi;
 *      * the polar condition eq. (3), which only defines the value reported at
 *        the poles (see orc_pole_values).
 *  - The discretization (Sec. 2.2): the second-order finite-difference
 *    Laplacian on a nonuniform (r, theta, phi) grid shown after eq. (3).  The
 *    unknowns sit at cell centres.  The printed scheme omits the spherical
 *    metric (r^2 on the radial faces, 1/r^2 on the angular terms).  It is
 *    used here with the metric restored, multiplied by the cell volume
 *    V = r_i^2 sin(theta_j) dr_i dtheta_j dphi_k and negated.  That gives the
 *    symmetric positive-definite matrix A that Sec. 2.3 calls for.  The
 *    paper keeps its boundary conditions out of the stored matrix (Sec. 2.2);
 *    here the surface data become the right-hand side b, so the matrix form
 *    A Phi = 0 of Sec. 2.2 reads A Phi = b.
 *  - The solver (Sec. 2.3): conjugate gradients preconditioned by the inverse
 *    of the diagonal of A ("PC1", point Jacobi), in the standard form of Saad's
 *    Algorithm 9.1.  The stopping test is ||r_k||_2 / ||b||_2 <= tol on the
 *    recursively updated residual (the relative tolerance of Sec. 4.1).
 *
 * Storage: A is kept as seven coefficient arrays of length N (the diagonal
 * and one weight per neighbour direction), the stencil form of the DIA storage
 * of Sec. 2.2.  The periodic phi neighbour wraps inside a row.  Index
 * P = (i*nt + j)*np + k, with phi fastest.
 *
 * Everything is plain IEEE double arithmetic with separate loops per
 * operation.  Dot products use Neumaier-compensated sums over a fixed
 * partition of the index range, so results do not depend on the thread count.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENOCONV (-4)
#define ORC_EBREAKDOWN (-5)

#define ORC_TWO_PI 6.283185307179586476925286766559

/* coefficient array order inside the 8*N block handed to orc_assemble */
enum { C_DIAG = 0, C_RM, C_RP, C_TM, C_TP, C_PM, C_PP, C_DTOP, C_COUNT };

static long idx3(int i, int j, int k, int nt, int np) { return ((long)i * nt + j) * np + k; }

/* ---------------------------------------------------------------------------
 * Operator assembly (Sec. 2.2 scheme, metric restored, times the cell volume).
 *
 * Cell c of a coordinate with faces f[0..n]: centre x_c = (f[c] + f[c+1]) / 2,
 * width w_c = f[c+1] - f[c], centre spacing x_{c+1} - x_c.  In phi the spacing
 * across the periodic seam is x_0 + 2 pi - x_{n-1}.
 *
 *   radial face i+1/2 (between centres i, i+1):
 *       W = dphi_k * sin(theta_j) dtheta_j * rf[i+1]^2 / (r_{i+1} - r_i)
 *   bottom face r = R0: no coupling (Neumann data go to b)
 *   top face r = R1, Phi = 0 on the face, one-sided difference over the half cell:
 *       Dtop = dphi_k * sin(theta_j) dtheta_j * rf[nr]^2 / (rf[nr] - r_{nr-1}), on the diagonal
 *       (closed wall, Br = 0 on the face: no flux, Dtop = 0)
 *   polar-angle face j+1/2:  W = dphi_k * dr_i * sin(tf[j+1]) / (theta_{j+1} - theta_j)
 *   pole faces (theta = 0, pi): sin = 0, so no coupling (set exactly to zero)
 *   azimuthal face k+1/2:    W = dr_i * dtheta_j / sin(theta_j) / (phi_{k+1} - phi_k)
 *   diagonal = sum of the neighbour weights present + Dtop
 * ------------------------------------------------------------------------- */
int orc_assemble_bc(const double *rf, int nr, const double *tf, int nt, const double *pf, int np, int closed_wall,
                    double *coef)
{
    if (nr < 1 || nt < 1 || np < 1 || !rf || !tf || !pf || !coef) return ORC_EINVAL;
    const long N = (long)nr * nt * np;
    double *rc = malloc(sizeof(double) * nr), *dr = malloc(sizeof(double) * nr);
    double *tc = malloc(sizeof(double) * nt), *dt = malloc(sizeof(double) * nt);
    double *pc = malloc(sizeof(double) * np), *dp = malloc(sizeof(double) * np);
    if (!rc || !dr || !tc || !dt || !pc || !dp) {
        free(rc); free(dr); free(tc); free(dt); free(pc); free(dp);
        return ORC_ENOMEM;
    }
    for (int i = 0; i < nr; i++) { rc[i] = 0.5 * (rf[i] + rf[i + 1]); dr[i] = rf[i + 1] - rf[i]; }
    for (int j = 0; j < nt; j++) { tc[j] = 0.5 * (tf[j] + tf[j + 1]); dt[j] = tf[j + 1] - tf[j]; }
    for (int k = 0; k < np; k++) { pc[k] = 0.5 * (pf[k] + pf[k + 1]); dp[k] = pf[k + 1] - pf[k]; }

    double *D = coef + C_DIAG * N, *WRM = coef + C_RM * N, *WRP = coef + C_RP * N;
    double *WTM = coef + C_TM * N, *WTP = coef + C_TP * N, *WPM = coef + C_PM * N;
    double *WPP = coef + C_PP * N, *DTOP = coef + C_DTOP * N;

    #pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; i++) {
        for (int j = 0; j < nt; j++) {
            for (int k = 0; k < np; k++) {
                const long P = idx3(i, j, k, nt, np);
                const double area_r = dp[k] * sin(tc[j]) * dt[j];   /* angular area of an r-face / r^2 */
                double wrm = 0.0, wrp = 0.0, wtm = 0.0, wtp = 0.0, dtop = 0.0;
                if (i > 0)      wrm = area_r * rf[i] * rf[i] / (rc[i] - rc[i - 1]);
                if (i < nr - 1) wrp = area_r * rf[i + 1] * rf[i + 1] / (rc[i + 1] - rc[i]);
                if (i == nr - 1 && !closed_wall) dtop = area_r * rf[nr] * rf[nr] / (rf[nr] - rc[nr - 1]);
                if (j > 0)      wtm = dp[k] * dr[i] * sin(tf[j]) / (tc[j] - tc[j - 1]);
                if (j < nt - 1) wtp = dp[k] * dr[i] * sin(tf[j + 1]) / (tc[j + 1] - tc[j]);
                double sp_minus = (k > 0) ? pc[k] - pc[k - 1] : pc[0] + ORC_TWO_PI - pc[np - 1];
                double sp_plus = (k < np - 1) ? pc[k + 1] - pc[k] : pc[0] + ORC_TWO_PI - pc[np - 1];
                double wpm = 0.0, wpp = 0.0;
                if (np > 1) {
                    const double area_p = dr[i] * dt[j] / sin(tc[j]);
                    wpm = area_p / sp_minus;
                    wpp = area_p / sp_plus;
                }
                WRM[P] = wrm; WRP[P] = wrp; WTM[P] = wtm; WTP[P] = wtp;
                WPM[P] = wpm; WPP[P] = wpp; DTOP[P] = dtop;
                D[P] = wrm + wrp + wtm + wtp + wpm + wpp + dtop;
            }
        }
    }
    free(rc); free(dr); free(tc); free(dt); free(pc); free(dp);
    return ORC_OK;
}

int orc_assemble(const double *rf, int nr, const double *tf, int nt, const double *pf, int np, double *coef)
{
    return orc_assemble_bc(rf, nr, tf, nt, pf, np, 0, coef);
}

/* y = A x: diagonal times the centre minus each neighbour weight times that
 * neighbour.  Neighbours outside the shell in r or across a pole do not exist
 * (their weights are zero); phi wraps. */
void orc_matvec(int nr, int nt, int np, const double *coef, const double *x, double *y)
{
    const long N = (long)nr * nt * np;
    const double *D = coef + C_DIAG * N, *WRM = coef + C_RM * N, *WRP = coef + C_RP * N;
    const double *WTM = coef + C_TM * N, *WTP = coef + C_TP * N, *WPM = coef + C_PM * N;
    const double *WPP = coef + C_PP * N;
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; i++) {
        for (int j = 0; j < nt; j++) {
            for (int k = 0; k < np; k++) {
                const long P = idx3(i, j, k, nt, np);
                double s = D[P] * x[P];
                if (i > 0)      s -= WRM[P] * x[idx3(i - 1, j, k, nt, np)];
                if (i < nr - 1) s -= WRP[P] * x[idx3(i + 1, j, k, nt, np)];
                if (j > 0)      s -= WTM[P] * x[idx3(i, j - 1, k, nt, np)];
                if (j < nt - 1) s -= WTP[P] * x[idx3(i, j + 1, k, nt, np)];
                if (np > 1) {
                    const int km = (k == 0) ? np - 1 : k - 1;
                    const int kp = (k == np - 1) ? 0 : k + 1;
                    s -= WPM[P] * x[idx3(i, j, km, nt, np)];
                    s -= WPP[P] * x[idx3(i, j, kp, nt, np)];
                }
                y[P] = s;
            }
        }
    }
}

/* Right-hand side: the surface condition eq. (2) as a flux through the r = R0
 * face of the first cell layer.  With dPhi/dr = -Br that flux, times -1 for the
 * negated operator, is  b = dphi_k sin(theta_j) dtheta_j R0^2 Br(j,k)  on i = 0,
 * and b = 0 elsewhere.  This is the finite-volume form of the paper's
 * ghost-cell fill (Sec. 3.5), which sets the ghost layer from Br times the
 * first radial spacing. */
void orc_rhs(const double *rf, int nr, const double *tf, int nt, const double *pf, int np,
             const double *br, double *b)
{
    const long N = (long)nr * nt * np;
    memset(b, 0, sizeof(double) * N);
    for (int j = 0; j < nt; j++) {
        const double tcj = 0.5 * (tf[j] + tf[j + 1]), dtj = tf[j + 1] - tf[j];
        for (int k = 0; k < np; k++) {
            const double dpk = pf[k + 1] - pf[k];
            b[idx3(0, j, k, nt, np)] = dpk * sin(tcj) * dtj * rf[0] * rf[0] * br[(long)j * np + k];
        }
    }
}

/* Closed wall: the shell then has no outlet, so the flux of B through r = R0
 * must vanish (Gauss's law for div B = 0), which is also the solvability
 * condition sum(b) = 0 of the singular system.  The surface data's monopole,
 * the area-weighted mean of Br over r = R0 (weights dphi_k sin(theta_j)
 * dtheta_j), is removed first; *mono receives it.  Data that are a monopole
 * up to rounding (the weighted 2-norm of Br - mean at most 1e-14 of that of
 * Br) give b = 0, so Phi = 0. */
void orc_rhs_bc(const double *rf, int nr, const double *tf, int nt, const double *pf, int np, int closed_wall,
                const double *br, double *b, double *mono)
{
    double m = 0.0, keep = 1.0;
    if (closed_wall) {
        double num = 0.0, den = 0.0;
        for (int j = 0; j < nt; j++) {
            const double tcj = 0.5 * (tf[j] + tf[j + 1]), dtj = tf[j + 1] - tf[j];
            for (int k = 0; k < np; k++) {
                const double w = (pf[k + 1] - pf[k]) * sin(tcj) * dtj;
                num += w * br[(long)j * np + k];
                den += w;
            }
        }
        m = num / den;
        double raw = 0.0, rest = 0.0;
        for (int j = 0; j < nt; j++) {
            const double tcj = 0.5 * (tf[j] + tf[j + 1]), dtj = tf[j + 1] - tf[j];
            for (int k = 0; k < np; k++) {
                const double w = (pf[k + 1] - pf[k]) * sin(tcj) * dtj;
                const double v = br[(long)j * np + k];
                raw += (w * v) * (w * v);
                rest += (w * (v - m)) * (w * (v - m));
            }
        }
        if (rest <= 1e-28 * raw) keep = 0.0;
    }
    if (mono) *mono = m;
    const long N = (long)nr * nt * np;
    memset(b, 0, sizeof(double) * N);
    for (int j = 0; j < nt; j++) {
        const double tcj = 0.5 * (tf[j] + tf[j + 1]), dtj = tf[j + 1] - tf[j];
        for (int k = 0; k < np; k++) {
            const double dpk = pf[k + 1] - pf[k];
            b[idx3(0, j, k, nt, np)] = keep * dpk * sin(tcj) * dtj * rf[0] * rf[0] * (br[(long)j * np + k] - m);
        }
    }
}

/* Closed wall: A Phi = b fixes Phi up to a constant.  The reported solution is
 * the one whose mean over the shell, weighted by the cell volumes
 * r_i^2 dr_i sin(theta_j) dtheta_j dphi_k, is zero. */
void orc_gauge(const double *rf, int nr, const double *tf, int nt, const double *pf, int np, double *x)
{
    double num = 0.0, den = 0.0;
    for (int i = 0; i < nr; i++) {
        const double rci = 0.5 * (rf[i] + rf[i + 1]), dri = rf[i + 1] - rf[i];
        for (int j = 0; j < nt; j++) {
            const double tcj = 0.5 * (tf[j] + tf[j + 1]), dtj = tf[j + 1] - tf[j];
            for (int k = 0; k < np; k++) {
                const double v = rci * rci * dri * sin(tcj) * dtj * (pf[k + 1] - pf[k]);
                num += v * x[idx3(i, j, k, nt, np)];
                den += v;
            }
        }
    }
    const double m = num / den;
    const long N = (long)nr * nt * np;
    for (long P = 0; P < N; P++) x[P] -= m;
}

/* The field B = -grad Phi (Sec. 2.1; the paper's B = grad Phi with our sign of
 * Phi) on the faces of the cells, by the same differences as the operator:
 *   Br on r-faces, (nr+1) x nt x np: -(Phi_i - Phi_{i-1}) / (r_i - r_{i-1})
 *      inside; the surface data br0 (Br less any removed monopole) on r = R0;
 *      on r = R1 Phi_{nr-1} / (R1 - r_{nr-1}) (Phi = 0 on the face), or 0 with
 *      the closed wall;
 *   Bt on theta-faces, nr x (nt+1) x np: -(Phi_j - Phi_{j-1}) / (r_i (theta_j - theta_{j-1}))
 *      inside, 0 on the pole faces;
 *   Bp on phi-faces k+1/2, nr x nt x np: -(Phi_{k+1} - Phi_k) / (r_i sin(theta_j) s_k),
 *      s_k the centre spacing (across the seam: phi_0 + 2 pi - phi_{np-1}).
 * With the face areas rf^2 sin(theta_j) dtheta_j dphi_k, r_i dr_i sin(tf_j) dphi_k and
 * r_i dr_i dtheta_j, the net outward flux of B from each cell is (A Phi - b) there. */
void orc_field(const double *rf, int nr, const double *tf, int nt, const double *pf, int np, int closed_wall,
               const double *br0, const double *x, double *bfr, double *bft, double *bfp)
{
    double *rc = malloc(sizeof(double) * nr), *tc = malloc(sizeof(double) * nt), *pc = malloc(sizeof(double) * np);
    if (!rc || !tc || !pc) {
        free(rc); free(tc); free(pc);
        return;
    }
    for (int i = 0; i < nr; i++) rc[i] = 0.5 * (rf[i] + rf[i + 1]);
    for (int j = 0; j < nt; j++) tc[j] = 0.5 * (tf[j] + tf[j + 1]);
    for (int k = 0; k < np; k++) pc[k] = 0.5 * (pf[k] + pf[k + 1]);
    for (int i = 0; i <= nr; i++)
        for (int j = 0; j < nt; j++)
            for (int k = 0; k < np; k++) {
                double v;
                if (i == 0) v = br0[(long)j * np + k];
                else if (i == nr) v = closed_wall ? 0.0 : x[idx3(nr - 1, j, k, nt, np)] / (rf[nr] - rc[nr - 1]);
                else v = -(x[idx3(i, j, k, nt, np)] - x[idx3(i - 1, j, k, nt, np)]) / (rc[i] - rc[i - 1]);
                bfr[((long)i * nt + j) * np + k] = v;
            }
    for (int i = 0; i < nr; i++)
        for (int j = 0; j <= nt; j++)
            for (int k = 0; k < np; k++) {
                double v = 0.0;
                if (j > 0 && j < nt)
                    v = -(x[idx3(i, j, k, nt, np)] - x[idx3(i, j - 1, k, nt, np)]) / (rc[i] * (tc[j] - tc[j - 1]));
                bft[((long)i * (nt + 1) + j) * np + k] = v;
            }
    for (int i = 0; i < nr; i++)
        for (int j = 0; j < nt; j++)
            for (int k = 0; k < np; k++) {
                const int kp = (k == np - 1) ? 0 : k + 1;
                const double sp = (k < np - 1) ? pc[k + 1] - pc[k] : pc[0] + ORC_TWO_PI - pc[np - 1];
                bfp[idx3(i, j, k, nt, np)] =
                    -(x[idx3(i, j, kp, nt, np)] - x[idx3(i, j, k, nt, np)]) / (rc[i] * sin(tc[j]) * sp);
            }
    free(rc); free(tc); free(pc);
}

/* ---- compensated dot over a fixed partition (deterministic for any thread count) */
#define ORC_CHUNKS 256

static void neumaier_add(double *sum, double *comp, double v)
{
    const double t = *sum + v;
    if (fabs(*sum) >= fabs(v)) *comp += (*sum - t) + v;
    else                       *comp += (v - t) + *sum;
    *sum = t;
}

double orc_dot(const double *a, const double *b, long n)
{
    double s[ORC_CHUNKS], c[ORC_CHUNKS];
    #pragma omp parallel for schedule(static)
    for (int t = 0; t < ORC_CHUNKS; t++) {
        const long lo = n * t / ORC_CHUNKS, hi = n * (t + 1) / ORC_CHUNKS;
        double sum = 0.0, comp = 0.0;
        for (long q = lo; q < hi; q++) neumaier_add(&sum, &comp, a[q] * b[q]);
        s[t] = sum;
        c[t] = comp;
    }
    double sum = 0.0, comp = 0.0;
    for (int t = 0; t < ORC_CHUNKS; t++) {
        neumaier_add(&sum, &comp, s[t]);
        neumaier_add(&sum, &comp, c[t]);
    }
    return sum + comp;
}

/* ---------------------------------------------------------------------------
 * phi-line Jacobi: a block preconditioner whose blocks are whole azimuthal
 * rows.  Sec. 2.3 uses the diagonal of A (PC1); its closing remarks (Sec. 6)
 * ask for other preconditioners that vectorize well.  Near the poles the
 * azimuthal weights (which carry 1 / sin(theta)) dwarf the radial and polar
 * ones, and the point-Jacobi diagonal cannot represent that coupling.
 *
 * M keeps, for every (i, j) row, the diagonal of A and its two azimuthal
 * neighbour weights (periodic in phi) and drops every coupling between rows.
 * Each block is symmetric and strictly diagonally dominant (the diagonal also
 * holds the radial and polar weights, and every cell has a radial
 * neighbour), so M is SPD and M^-1 exists.
 *
 * z = M^-1 r is one periodic tridiagonal solve per row.  For a row of n >= 3
 * cells with diagonal d_k, lower weight a_k = W_phi-(k) and upper weight
 * c_k = W_phi+(k):
 *     d_k z_k - a_k z_{k-1} - c_k z_{k+1} = r_k      (indices mod n)
 * The two corner entries (-a_0 in row 0, -c_{n-1} in row n-1) are split off
 * as a rank-one term u v^T with u = (g, 0, .., 0, -c_{n-1}),
 * v = (1, 0, .., 0, -a_0 / g) and g = -d_0, leaving a tridiagonal T whose
 * first and last diagonal entries are d_0 - g and d_{n-1} - c_{n-1} a_0 / g.
 * The Sherman-Morrison formula then gives
 *     z = y - (v.y / (1 + v.q)) q,   T y = r,   T q = u,
 * and both solves with T are plain Thomas eliminations sharing one forward
 * sweep.  n = 1 has no azimuthal coupling (z = r / d); for n = 2 both
 * neighbours are the other cell and the 2 x 2 block is solved directly.
 * ------------------------------------------------------------------------- */
int orc_line_solve(int nr, int nt, int np, const double *coef, const double *r, double *z)
{
    const long N = (long)nr * nt * np;
    const double *D = coef + C_DIAG * N, *WPM = coef + C_PM * N, *WPP = coef + C_PP * N;
    const long rows = (long)nr * nt;
    int status = ORC_OK;
    #pragma omp parallel
    {
        double *cp = malloc(sizeof(double) * (np > 0 ? np : 1));
        double *y = malloc(sizeof(double) * (np > 0 ? np : 1));
        double *q = malloc(sizeof(double) * (np > 0 ? np : 1));
        if (!cp || !y || !q) {
            #pragma omp atomic write
            status = ORC_ENOMEM;
        }
        #pragma omp for schedule(static)
        for (long row = 0; row < rows; row++) {
            if (!cp || !y || !q) continue;
            const long o = row * np;
            const double *d = D + o, *a = WPM + o, *c = WPP + o, *rr = r + o;
            double *zz = z + o;
            if (np == 1) {
                zz[0] = rr[0] / d[0];
                continue;
            }
            if (np == 2) {
                const double m01 = -(a[0] + c[0]), m10 = -(a[1] + c[1]);
                const double det = d[0] * d[1] - m01 * m10;
                zz[0] = (d[1] * rr[0] - m01 * rr[1]) / det;
                zz[1] = (d[0] * rr[1] - m10 * rr[0]) / det;
                continue;
            }
            const int n = np;
            const double g = -d[0];
            /* forward sweep of T for both right-hand sides r and u */
            double w = d[0] - g;
            cp[0] = -c[0] / w;
            y[0] = rr[0] / w;
            q[0] = g / w;
            for (int k = 1; k < n; k++) {
                double dk = d[k];
                if (k == n - 1) dk -= c[n - 1] * a[0] / g;
                const double lk = -a[k];
                w = dk - lk * cp[k - 1];
                cp[k] = (k < n - 1) ? -c[k] / w : 0.0;
                const double uk = (k == n - 1) ? -c[n - 1] : 0.0;
                y[k] = (rr[k] - lk * y[k - 1]) / w;
                q[k] = (uk - lk * q[k - 1]) / w;
            }
            for (int k = n - 2; k >= 0; k--) {
                y[k] -= cp[k] * y[k + 1];
                q[k] -= cp[k] * q[k + 1];
            }
            const double vy = y[0] - (a[0] / g) * y[n - 1];
            const double vq = q[0] - (a[0] / g) * q[n - 1];
            const double f = vy / (1.0 + vq);
            for (int k = 0; k < n; k++) zz[k] = y[k] - f * q[k];
        }
        free(cp); free(y); free(q);
    }
    return status;
}

/* ---------------------------------------------------------------------------
 * Jacobi-preconditioned CG (Sec. 2.3; Saad, Algorithm 9.1 with M = diag(A)).
 *
 *   x = x0; r = b - A x; z = r / d; p = z; rho = r.z
 *   for k = 1 .. maxit:
 *       q = A p; sigma = p.q          (sigma <= 0 or not finite: breakdown)
 *       alpha = rho / sigma; x += alpha p; r -= alpha q
 *       stop when ||r|| / ||b|| <= tol (iters = k)
 *       z = r / d; rho' = r.z; beta = rho' / rho; rho = rho'; p = z + beta p
 *
 * x holds x0 on entry (zeros for a cold start) and the last iterate on exit.
 * ||b|| = 0 gives x = 0, iters = 0.  A start that already meets tol returns
 * iters = 0.  Non-finite data give ORC_EBREAKDOWN with the last finite
 * iterate.  tol = 0 runs exactly maxit iterations (fixed-count mode).
 * ------------------------------------------------------------------------- */
/* The preconditioner of orc_pcg_pc: the diagonal of A (PC1, Sec. 2.3), or the
 * phi-line blocks of orc_line_solve. */
#define ORC_PC_JACOBI 0
#define ORC_PC_PHI_LINE 1

static int precondition(int precond, int nr, int nt, int np, const double *coef, const double *r, double *z)
{
    const long N = (long)nr * nt * np;
    if (precond == ORC_PC_PHI_LINE) return orc_line_solve(nr, nt, np, coef, r, z);
    const double *D = coef + C_DIAG * N;
    #pragma omp parallel for schedule(static)
    for (long P = 0; P < N; P++) z[P] = r[P] / D[P];
    return ORC_OK;
}

int orc_pcg_pc(int nr, int nt, int np, const double *coef, const double *b, double *x,
               double tol, int maxit, int precond, int *iters_out, double *relres_out);

int orc_pcg(int nr, int nt, int np, const double *coef, const double *b, double *x,
            double tol, int maxit, int *iters_out, double *relres_out)
{
    return orc_pcg_pc(nr, nt, np, coef, b, x, tol, maxit, ORC_PC_JACOBI, iters_out, relres_out);
}

/* The same PCG with z = M^-1 r from the chosen preconditioner. */
int orc_pcg_pc(int nr, int nt, int np, const double *coef, const double *b, double *x,
               double tol, int maxit, int precond, int *iters_out, double *relres_out)
{
    const long N = (long)nr * nt * np;
    double *r = malloc(sizeof(double) * N), *z = malloc(sizeof(double) * N);
    double *p = malloc(sizeof(double) * N), *q = malloc(sizeof(double) * N);
    int status = ORC_OK, iters = 0;
    double relres = 0.0;
    if (!r || !z || !p || !q) { status = ORC_ENOMEM; goto done; }

    const double nb = sqrt(orc_dot(b, b, N));
    if (!isfinite(nb)) { status = ORC_EBREAKDOWN; relres = NAN; goto done; }
    if (nb == 0.0) {
        memset(x, 0, sizeof(double) * N);
        goto done;
    }
    orc_matvec(nr, nt, np, coef, x, q);
    #pragma omp parallel for schedule(static)
    for (long P = 0; P < N; P++) r[P] = b[P] - q[P];
    relres = sqrt(orc_dot(r, r, N)) / nb;
    if (!isfinite(relres)) { status = ORC_EBREAKDOWN; goto done; }
    if (relres <= tol) goto done;

    if (precondition(precond, nr, nt, np, coef, r, z) != ORC_OK) { status = ORC_ENOMEM; goto done; }
    #pragma omp parallel for schedule(static)
    for (long P = 0; P < N; P++) p[P] = z[P];
    double rho = orc_dot(r, z, N);

    status = ORC_ENOCONV;
    for (int k = 1; k <= maxit; k++) {
        orc_matvec(nr, nt, np, coef, p, q);
        const double sigma = orc_dot(p, q, N);
        if (!(sigma > 0.0) || !isfinite(sigma)) { status = ORC_EBREAKDOWN; break; }
        const double alpha = rho / sigma;
        #pragma omp parallel for schedule(static)
        for (long P = 0; P < N; P++) { x[P] += alpha * p[P]; r[P] -= alpha * q[P]; }
        iters = k;
        relres = sqrt(orc_dot(r, r, N)) / nb;
        if (!isfinite(relres)) { status = ORC_EBREAKDOWN; break; }
        if (relres <= tol) { status = ORC_OK; break; }
        if (precondition(precond, nr, nt, np, coef, r, z) != ORC_OK) { status = ORC_ENOMEM; break; }
        const double rho_new = orc_dot(r, z, N);
        const double beta = rho_new / rho;
        rho = rho_new;
        #pragma omp parallel for schedule(static)
        for (long P = 0; P < N; P++) p[P] = z[P] + beta * p[P];
    }
done:
    free(r); free(z); free(p); free(q);
    if (iters_out) *iters_out = iters;
    if (relres_out) *relres_out = relres;
    return status;
}

/* ||b - A x||_2 / ||b||_2 (the true relative residual). */
double orc_true_relres(int nr, int nt, int np, const double *coef, const double *b, const double *x)
{
    const long N = (long)nr * nt * np;
    double *q = malloc(sizeof(double) * N);
    if (!q) return NAN;
    orc_matvec(nr, nt, np, coef, x, q);
    #pragma omp parallel for schedule(static)
    for (long P = 0; P < N; P++) q[P] = b[P] - q[P];
    const double num = sqrt(orc_dot(q, q, N)), den = sqrt(orc_dot(b, b, N));
    free(q);
    return num / den;
}

/* Pole values, eq. (3): the phi-average of Phi on the ring of cell centres
 * half a pole cell away from the pole (j = 0 for theta = 0, j = nt-1 for
 * theta = pi), one value per radial layer:
 *   Phi_pole(i) = (1 / 2 pi) sum_k dphi_k Phi(i, ring, k). */
void orc_pole_values(int nr, int nt, int np, const double *pf, const double *x, double *north, double *south)
{
    const double span = pf[np] - pf[0];
    for (int i = 0; i < nr; i++) {
        double sn = 0.0, ss = 0.0;
        for (int k = 0; k < np; k++) {
            const double dpk = pf[k + 1] - pf[k];
            sn += dpk * x[idx3(i, 0, k, nt, np)];
            ss += dpk * x[idx3(i, nt - 1, k, nt, np)];
        }
        north[i] = sn / span;
        south[i] = ss / span;
    }
}

/* OpenMP threads of the following calls (timing runs of the benchmark's CPU
 * baseline: one thread as in the paper's serial baseline, Sec. 4.1, or all);
 * returns the number the runtime will use. */
int orc_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}
