/*
 * pot3d.h -- C ABI of the MI355X potential-field solver.
 *
 * The library solves Laplace's equation for the magnetic potential Phi on a
 * spherical shell 1 = R0 <= r <= R1 (Caplan, Mikic & Linker,
 * arXiv:1709.01126, Sec. 2.1, eq. (1)).  The boundary conditions are:
 *   * r = R0: the surface condition eq. (2), read as dPhi/dr = -Br, so that
 *     B = -grad Phi.  The paper writes B = +grad Phi with dPhi/dr = +Br; its
 *     potential is the negative of the one returned here;
 *   * r = R1: the "source surface" Phi = 0 (Sec. 2.1);
 *   * phi: periodic;
 *   * poles: eq. (3) only defines the value reported there, see
 *     pot3d_pole_values.
 *
 * Discretization (Sec. 2.2): the second-order finite-difference Laplacian on
 * a nonuniform, logically rectangular (r, theta, phi) grid, with unknowns at
 * cell centres.  It is used in its symmetric finite-volume form: spherical
 * metric restored, scaled by the cell volume, negated.  That gives the
 * symmetric positive-definite system A Phi = b, where b carries the surface
 * flux of Br.
 *
 * Solver (Sec. 2.3): conjugate gradients with the point-Jacobi
 * preconditioner (the inverse of the diagonal of A, "PC1").  It stops when
 * ||r_k||_2 / ||b||_2 <= tol on the recursively updated residual, the
 * relative tolerance of Sec. 4.1.
 *
 * Layouts: every 3-D array is C order with phi fastest,
 *     a[(i*nt + j)*np + k],  i radial, j polar (from theta = 0), k azimuthal,
 * and every surface map is br[j*np + k], sampled at the angular cell centres.
 *
 * Ownership: the caller owns every buffer passed in.  The library copies the
 * faces at create time and reads Br and Phi0 during a call only.  It keeps
 * all of its device memory in the context until pot3d_destroy.
 *
 * Errors: every int-returning call returns a POT3D_* status.  Argument
 * checks run before any device call, so POT3D_EINVAL paths work without a
 * GPU.  pot3d_last_error gives a readable message.  A context is not
 * thread-safe; distinct contexts may be used from different threads.
 */
#ifndef POT3D_H
#define POT3D_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pot3d_ctx pot3d_ctx;

enum pot3d_status {
    POT3D_OK = 0,
    POT3D_EINVAL = -1,      /* bad argument; nothing was done                           */
    POT3D_ENOMEM = -2,      /* device or host allocation failed                         */
    POT3D_EDEVICE = -3,     /* HIP runtime error (no device, launch failure, ...)       */
    POT3D_ENOCONV = -4,     /* maxit reached; Phi, iters, relres hold the last iterate  */
    POT3D_EBREAKDOWN = -5   /* non-finite data or p.Ap <= 0; the last finite iterate
                               is returned                                             */
};

enum pot3d_upper_bc {
    POT3D_UPPER_SOURCE_SURFACE = 0,   /* Phi(R1) = 0 (Sec. 2.1)                                   */
    POT3D_UPPER_CLOSED_WALL = 1       /* Br(R1) = 0 (Sec. 2.1): no flux through the top face.  The
                                         system is singular (constants); the area-weighted mean of
                                         Br (its monopole, which a closed shell cannot carry) is
                                         removed from b, data that are a monopole up to rounding
                                         give Phi = 0, and Phi is returned with zero mean weighted
                                         by the cell volumes.  Single solves only (not the server). */
};

enum pot3d_refine_mode {
    POT3D_REFINE_RESTART = 0,   /* each inner FP32 solve starts a fresh PCG (p = 0)             */
    POT3D_REFINE_RELIABLE = 1   /* each inner solve continues the previous one's search
                                   direction after the FP64 residual replacement (default)     */
};

enum pot3d_iteration {
    POT3D_ITER_TWO_PASS = 0,   /* two sweeps over memory per PCG iteration: the direction
                                  update with A p and p.Ap, then the r/x update with r.z and
                                  r.r; x once per pair of iterations (the odd r/x update
                                  reads p_{k-1}): 60 bytes per unknown on average, 64 with
                                  POT3D_SWEEP_X=1                                             */
    POT3D_ITER_ONE_SWEEP = 1   /* one sweep per iteration: the r/x update of iteration j-1
                                  and the direction update of iteration j together, with
                                  r.z of the next residual predicted from p.Ap, z.Ap and
                                  Ap.D^-1 Ap.  x is updated once per pair of sweeps, the
                                  earlier increment rebuilt from p and z: 40 bytes per
                                  unknown per iteration in FP64, 20 in FP32 (48 and 24
                                  with POT3D_SWEEP_X=1 in the environment, x every sweep).
                                  The same PCG in exact arithmetic.  Default.               */
};

enum pot3d_preconditioner {
    POT3D_PC_JACOBI = 0,     /* point Jacobi, M = diag(A): "PC1" of Sec. 2.3 (default)       */
    POT3D_PC_PHI_LINE = 1    /* phi-line blocks: M keeps, for every (r, theta) row, the
                                diagonal of A and its two periodic azimuthal weights and
                                drops the couplings between rows; z = M^-1 r is one
                                periodic tridiagonal solve per row.  A stronger
                                preconditioner of the kind Sec. 6 calls for: near the poles
                                the azimuthal weights, which carry 1 / sin(theta), dominate
                                the diagonal, and point Jacobi cannot represent them.       */
};

enum pot3d_precision {
    POT3D_FP64 = 0,          /* FP64 vectors, stencil and reductions throughout              */
    POT3D_FP32_REFINED = 1   /* FP32 inner PCG inside FP64 defect correction (see
                                pot3d_solve_device)                                        */
};

typedef struct pot3d_stats {
    int iters;               /* PCG iterations of the last solve (inner iterations summed
                                in refined mode)                                           */
    int outer;               /* defect-correction cycles (1 in FP64 mode)                    */
    int status;              /* status of the last solve                                    */
    int graph_launches;      /* replays of the captured iteration graph                     */
    double relres;           /* recursive ||r||/||b|| at exit (FP64 mode)                   */
    double relres_true;      /* ||b - A Phi||/||b||, recomputed in FP64 at exit             */
    double solve_ms;         /* wall time of the last solve call on the device             */
    double loop_ms;          /* device time of the iteration loop (hipEvents)               */
    double bytes_per_iter;   /* algorithmic HBM bytes of one iteration, x once per pair of
                                iterations (with POT3D_SWEEP_X=1, x every iteration): FP64
                                40 N (48 N) one sweep, 60 N (64 N) two passes, 76 N (80 N)
                                with the phi-line preconditioner; FP32 inner iterations
                                half of each                                               */
    long long n;             /* unknowns nr*nt*np                                            */
    int pitch;               /* row pitch (elements) of the internal phi-fastest arrays    */
    int tile_p, tile_r;      /* stencil kernel shape of the p update and of the r/x update:
                                8/16/32 = workgroup tile of that many polar rows x 64
                                cells; 102/104/108 = wavefront tile of 2/4/8 rows x 128   */
    int chunk_p, chunk_r;    /* radial layers per workgroup chunk, per pass                 */
    int blocks_p, blocks_r;  /* workgroups per launch, per pass                              */
    int iteration;           /* POT3D_ITER_* of the iterations (FP32 inner ones if refined) */
    int sweep_rows;          /* one-sweep kernel: tile box rows per wavefront (4, 6 or 8)   */
    int chunk_s, blocks_s;   /* one-sweep kernel: radial layers per chunk, workgroups      */
    int precond;             /* POT3D_PC_* of the last solve                               */
    int blocks_l;            /* workgroups of the phi-line pass (0 unless POT3D_PC_PHI_LINE)*/
} pot3d_stats;

/*
 * Create a solver context for one grid (Sec. 2.2 mesh), on HIP device `device`.
 *   r_faces[0..nr]   strictly increasing, r_faces[0] > 0 (R0 = r_faces[0], R1 = r_faces[nr])
 *   t_faces[0..nt]   strictly increasing polar faces, t_faces[0] = 0, t_faces[nt] = pi
 *   p_faces[0..np]   strictly increasing azimuthal faces, p_faces[np] - p_faces[0] = 2 pi
 *   nr >= 2, nt >= 2, np >= 3.  Arrays are host memory, copied.
 *   upper_bc   POT3D_UPPER_SOURCE_SURFACE or POT3D_UPPER_CLOSED_WALL
 *   precision  POT3D_FP64 or POT3D_FP32_REFINED
 * On success *out owns device buffers of about 40 N bytes (FP64) or 32 N + 20 N
 * bytes (FP32-refined).
 */
int pot3d_create(const double *r_faces, int nr,
                 const double *t_faces, int nt,
                 const double *p_faces, int np,
                 int upper_bc, int precision, int device, pot3d_ctx **out);

/*
 * Solve A Phi = b(Br) from host memory (Sec. 2.1-2.3).
 *   br     host, nt*np, br[j*np + k]: Br at the angular cell centres of r = R0
 *   tol    >= 0; stop when ||r||/||b|| <= tol; tol = 0 runs exactly maxit iterations
 *   maxit  >= 0 iteration cap
 *   phi0   host, N, initial guess; NULL starts from zero
 *   phi    host, N, out: the solution (also filled on ENOCONV / EBREAKDOWN)
 *   iters  out (may be NULL): iterations performed
 *   relres_true out (may be NULL): ||b - A Phi||_2 / ||b||_2 recomputed at exit
 * Includes the host<->device copies of Br, Phi0 and Phi.
 */
int pot3d_solve(pot3d_ctx *ctx, const double *br, double tol, int maxit,
                const double *phi0, double *phi, int *iters, double *relres_true);

/*
 * As pot3d_solve, with device buffers and the caller's HIP stream
 * (hipStream_t passed as void*; NULL = the context's own stream).
 *   d_br   device, nt*np;  d_phi0 device, N or NULL;  d_phi device, N, out.
 * All work is ordered on `stream`; the call returns after the solve has
 * finished (it waits on the stream for the convergence flag).
 * In POT3D_FP32_REFINED contexts the outer loop recomputes r = b - A Phi in
 * FP64, runs FP32 PCG iterations on A e = r / ||r|| until their residual has
 * dropped by inner_tol, and adds ||r|| e to Phi in FP64 (see
 * pot3d_set_refinement_mode).  It repeats until the FP64 true residual is
 * <= tol.
 */
int pot3d_solve_device(pot3d_ctx *ctx, const double *d_br, const double *d_phi0, double *d_phi,
                       void *stream, double tol, int maxit, int *iters, double *relres_true);

/*
 * y = A x with the solver's own stencil (the Sec. 2.2 operator, volume-scaled).
 * d_x, d_y: device, N each, phi-fastest, distinct.  Ordered on `stream`
 * (NULL = the context's stream); returns after the kernel has completed.
 */
int pot3d_apply_device(pot3d_ctx *ctx, const double *d_x, double *d_y, void *stream);

/*
 * z = M^-1 r with the context's preconditioner (pot3d_set_preconditioner:
 * point Jacobi, the diagonal of A, Sec. 2.3; or the phi-line blocks).
 * d_r, d_z: device, N each, phi-fastest, distinct.  FP64 contexts only
 * (POT3D_EINVAL otherwise).  Ordered on `stream` (NULL = the context's);
 * returns after the kernel has completed.
 */
int pot3d_precondition_device(pot3d_ctx *ctx, const double *d_r, double *d_z, void *stream);

/*
 * Right-hand side b (device, N): the surface flux of Br through the r = R0
 * faces on the first radial layer, zero elsewhere (eq. (2) as a boundary flux);
 * with the closed wall, of Br less its monopole.
 */
int pot3d_rhs_device(pot3d_ctx *ctx, const double *d_br, double *d_b, void *stream);

/*
 * Pole values of the last solution, eq. (3): for each radial layer, the
 * phi-average of Phi on the ring of cell centres half a pole cell from the
 * pole.  north, south: host, nr each.
 */
int pot3d_pole_values(const pot3d_ctx *ctx, double *north, double *south);

/*
 * The field of the last solution, B = -grad Phi (Sec. 2.1; the paper writes
 * B = grad Phi for the opposite sign of Phi), on the cell faces by the
 * scheme's own differences, device buffers, phi fastest:
 *   d_br  (nr+1)*nt*np  Br on the r-faces i = 0..nr: the surface data on R0
 *         (less the monopole with the closed wall), Phi / half-cell on R1
 *         (0 with the closed wall);
 *   d_bt  nr*(nt+1)*np  Btheta on the theta-faces j = 0..nt (0 on the poles);
 *   d_bp  nr*nt*np      Bphi on the phi-faces k+1/2 (periodic).
 * With the face areas of the scheme, the net outward flux of B from each cell
 * is the residual (A Phi - b) there.  Ordered on `stream` (NULL = the
 * context's), returns when done.  POT3D_EINVAL before a solve, or after
 * pot3d_rhs_device or pot3d_time_kernels.
 */
int pot3d_field_device(pot3d_ctx *ctx, double *d_br, double *d_bt, double *d_bp, void *stream);

/* Statistics of the last solve. */
int pot3d_get_stats(const pot3d_ctx *ctx, pot3d_stats *out);

/*
 * Benchmark helper: average duration in ms of the per-iteration stencil
 * kernels as they run in a solve: a graph of `reps` iterations in the
 * solve's order is replayed twice back to back on the context's stream, and
 * in the second replay each stencil launch records its first workgroup's
 * start and its last workgroup's end on the device wall clock.
 * Two-pass iteration: *ms_update_p = the p update (A p, p.Ap), *ms_update_r =
 * the r/x update (r.z, r.r).  One-sweep iteration: *ms_update_p = the even
 * sweeps (x left to the next sweep), *ms_update_r = the odd sweeps (x of the
 * pair); with POT3D_SWEEP_X=1 both time the sweep that updates x every time.
 * FP32-refined contexts time the FP32 inner kernels.  It runs on the vectors
 * the context holds and overwrites them; a later solve re-initializes
 * everything.
 */
int pot3d_time_kernels(pot3d_ctx *ctx, int reps, double *ms_update_p, double *ms_update_r);

/*
 * FP32-refined contexts only: tolerance of each inner FP32 solve, relative to
 * its right-hand side ||r||, in (0, 1), and the most outer defect-correction
 * cycles (default 50).  Default tolerance: 0.1 in reliable-update mode, 1e-4
 * in restart mode (a reliable update every 1e-3 lets the FP32 recursion drift
 * and can take many times the iterations).  POT3D_EINVAL otherwise.
 */
int pot3d_set_refinement(pot3d_ctx *ctx, double inner_tol, int max_outer);

/*
 * FP32-refined contexts only: how an inner FP32 solve starts after the FP64
 * residual r = b - A Phi has been recomputed and Phi corrected.
 *   POT3D_REFINE_RESTART   a fresh PCG on r / ||r|| (plain defect correction);
 *   POT3D_REFINE_RELIABLE  r / ||r|| replaces the FP32 recursive residual, and
 *                          the last search direction (rescaled) and the beta
 *                          recurrence continue: residual replacement as in the
 *                          reliable-update CG of Sleijpen and van der Vorst.
 *                          A continued segment is capped at twice the
 *                          iterations of the one before (plus 64); after a
 *                          segment that did not converge the next one
 *                          restarts.  Default.
 * POT3D_EINVAL for other contexts or modes.
 */
int pot3d_set_refinement_mode(pot3d_ctx *ctx, int mode);

/*
 * The form of the PCG iteration: of the FP64 iterations, or in FP32-refined
 * contexts of the FP32 inner iterations (POT3D_ITER_ONE_SWEEP or
 * POT3D_ITER_TWO_PASS).  Default: one sweep, except for FP32-refined contexts
 * whose FP64 vectors reach 512 MiB, where the FP32 passes stream faster in
 * two; the environment variable POT3D_ITERATION = 0 or 1 sets the default of
 * new contexts (and the form of a batching server when it is created).  Both run the Jacobi-PCG of Sec. 2.3;
 * their iterates agree to rounding.  The one-sweep form needs vectors under
 * 4 GiB (FP64: N < 2^29 with the row padding); larger contexts accept
 * POT3D_ITER_TWO_PASS only.  POT3D_EINVAL otherwise.
 */
int pot3d_set_iteration(pot3d_ctx *ctx, int iteration);

/*
 * Preconditioner of the context's PCG iterations: the FP64 iterations of an
 * FP64 context, or the FP32 inner iterations of an FP32-refined one (Sec. 2.3
 * uses point Jacobi; Sec. 6 asks for stronger ones that still suit vector
 * hardware):
 *   POT3D_PC_JACOBI    point Jacobi (default), either iteration form;
 *   POT3D_PC_PHI_LINE  phi-line blocks.  Each PCG iteration then runs the
 *                      direction update on z = M^-1 r, the r/x update, and a
 *                      line pass that solves the rows (one wavefront per row:
 *                      the circulant block of a uniform phi grid factors
 *                      into two first-order periodic recurrences, always
 *                      evaluated in FP64) and writes z: 76 bytes per unknown
 *                      per FP64 iteration (38 per FP32 one) against 40 or 60
 *                      for point Jacobi, for fewer iterations.  Allocates one
 *                      more vector (8 N or 4 N bytes) on first use.
 * POT3D_EINVAL (nothing changed) unless the context's phi faces are uniform
 * (every width 2 pi / np to 1e-12 relative) with np <= 2048, or for another
 * value of pc.  POT3D_ENOMEM / POT3D_EDEVICE if the vector or the iteration
 * graph cannot be made.
 */
int pot3d_set_preconditioner(pot3d_ctx *ctx, int pc);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): the FP64
 * point-Jacobi solve of pot3d_create + pot3d_solve_device + pot3d_destroy in
 * one call that allocates nothing.  It runs the same one-sweep kernels; every
 * buffer beyond the arguments (metric tables, b layer, x, r, p, partial sums,
 * scalars) lives in a fixed 96 MiB device array that the library holds on
 * each GPU it runs on until the process ends.
 *   faces, upper_bc  as in pot3d_create (host arrays, read during the call)
 *   d_br    device, nt*np;  d_phi0 device, N or NULL;  d_phi device, N, out
 *   stream  hipStream_t as void* (NULL: the null stream); the work runs on the
 *           current device, and the call returns when it is done
 *   tol, maxit, iters, relres_true  as in pot3d_solve_device
 * Limits: nr, nt, np <= 4096, nr*nt <= 65536, and 40 bytes per padded cell
 * plus the tables within 96 MiB (64 x 128 x 256 fits; 101 x 201 x 401 does
 * not): POT3D_EINVAL, before any device work, beyond them.  Calls are
 * serialized by a process-wide lock (the array is shared by every call on a
 * GPU and keeps the last call's contents); each call clears what must start
 * at zero.  Returns the solve status as pot3d_solve_device does.
 */
int pot3d_solve_noalloc(const double *r_faces, int nr, const double *t_faces, int nt, const double *p_faces, int np,
                        int upper_bc, const double *d_br, const double *d_phi0, double *d_phi, void *stream,
                        double tol, int maxit, int *iters, double *relres_true);

/* Free the context and all of its device memory.  NULL is a no-op. */
void pot3d_destroy(pot3d_ctx *ctx);

/* Message of the last error on ctx (ctx = NULL: the calling thread's last
 * create/validation error).  Never NULL; valid until the next call. */
const char *pot3d_last_error(const pot3d_ctx *ctx);

/* Library version string. */
const char *pot3d_version(void);

/* ------------------------------------------------------------------------
 * Continuous-batching server.
 *
 * Many independent solves, each one the problem of Sec. 2.1-2.3 on its own
 * grid with its own surface map Br, share the GPU.  Requests queue on the
 * host.  Each pot3d_server_step:
 *   1. retires the solves that ended in the previous step;
 *   2. admits queued requests, in order, while a slot is free, their device
 *      memory fits the budget, and the bytes that the active solves stream
 *      per iteration stay within the cache budget (or no solve is active);
 *      a request that does not fit beside the active solves may be passed
 *      by up to 8 later ones that do, then waits at the head;
 *   3. advances every active solve by a fixed number of PCG iterations
 *      (32 sweeps in the one-sweep form, 16 two-pass iterations otherwise;
 *      the form is POT3D_ITERATION's when the server is created, one sweep
 *      by default), all in one replay of one captured HIP graph.
 * As in Sec. 3.1, the vectors of a solve stay in device memory from
 * admission to retirement.  Device memory per grid (tables and vectors) is
 * cached and reused by later requests on the same grid.  A solve that has
 * converged stops iterating at once, while the others go on.  Every result
 * is bitwise the one pot3d_solve gives for the same request on a context of
 * the same precision, iteration form and the default launch shape, for grids
 * whose vectors are below 512 MiB (above that, pot3d_solve switches to a
 * shape for HBM-streaming grids, which the server does not use).  Requests
 * take the source-surface upper boundary.  In the one-sweep form a request
 * whose grid needs vectors of 4 GiB or more finishes with POT3D_EINVAL.
 * ------------------------------------------------------------------------ */
typedef struct pot3d_server pot3d_server;

typedef struct pot3d_request_info {
    long long id;
    int done;                /* 1 once the request has left the server          */
    int status;              /* POT3D_* status of the solve (valid when done)   */
    int iters;               /* PCG iterations (inner iterations summed in
                                refined mode)                                   */
    int outer;               /* defect-correction cycles (1 in FP64 mode)        */
    int nr, nt, np;
    double relres_true;      /* ||b - A Phi||/||b|| recomputed in FP64 at exit  */
    double t_submit, t_admit, t_done;   /* seconds since server creation; -1 if
                                           not reached                         */
} pot3d_request_info;

typedef struct pot3d_server_stats {
    long long replays;       /* graph replays so far                            */
    long long finished;      /* requests done (solved or failed)                */
    int active, queued;      /* requests in slots and waiting                   */
    int cached_contexts;     /* idle per-grid device contexts held for reuse    */
    int max_slots;
    int graph_iters;         /* PCG iterations per replay                       */
    double used_bytes;       /* device bytes held by contexts (active + cached) */
    double budget_bytes;
} pot3d_server_stats;

/*
 * Create a server on `device`.
 *   precision         POT3D_FP64 or POT3D_FP32_REFINED, for all requests
 *   max_slots         1..64 concurrent solves
 *   hbm_budget_bytes  device bytes the per-grid contexts may hold; 0 = 80% of
 *                     the free device memory at creation
 * Allocates the slot tables and captures the batched graph.
 */
int pot3d_server_create(int device, int precision, int max_slots, double hbm_budget_bytes,
                        pot3d_server **out);

/*
 * Queue one solve.  Faces, nr, nt, np and br as in pot3d_create and
 * pot3d_solve (host memory, copied); tol and maxit as in pot3d_solve.
 * phi_out: host, nr*nt*np, where the server writes Phi when the solve
 * retires (it must stay valid until the request is done), or NULL to let the
 * server keep Phi until pot3d_server_result.  *id receives the request id.
 * Only validates and copies; no device work.
 */
int pot3d_server_submit(pot3d_server *sv, const double *r_faces, int nr, const double *t_faces, int nt,
                        const double *p_faces, int np, const double *br, double tol, int maxit,
                        double *phi_out, long long *id);

/*
 * One scheduling step (retire, admit, one graph replay); returns after the
 * replay has finished.  Out (each may be NULL): active slots, queued requests,
 * and requests finished so far.  A request that cannot run on this server (a
 * grid whose launch does not fit a slot, or whose context cannot be
 * allocated) finishes with that error status and no Phi.
 */
int pot3d_server_step(pot3d_server *sv, int *n_active, int *n_queued, long long *n_finished);

/*
 * State of request `id` into *info (may be NULL).  Once it is done and phi is
 * not NULL, Phi (host, nr*nt*np, phi-fastest) is copied into phi (no copy if
 * phi is the submit-time phi_out, which already holds it) and the request is
 * forgotten; later calls with its id return POT3D_EINVAL.
 */
int pot3d_server_result(pot3d_server *sv, long long id, double *phi, pot3d_request_info *info);

/*
 * Streaming budget of the batch: a request joins the active solves only if
 * the bytes they all stream per iteration (32 per cell in FP64, 16 in refined
 * mode) stay within `bytes`, or if none is active.  Default 256 MiB, the
 * memory-side cache of the device: solves that run from it alone are not
 * slowed by batching, and bandwidth-bound ones run alone, since batching
 * cannot speed them up.  0 removes the limit.
 */
int pot3d_server_set_cache_budget(pot3d_server *sv, double bytes);

int pot3d_server_get_stats(const pot3d_server *sv, pot3d_server_stats *out);

/* Waits for the device, then frees every context and the server.  NULL is a no-op. */
void pot3d_server_destroy(pot3d_server *sv);

/* Message of the last error on sv (sv = NULL: the thread's last create error). */
const char *pot3d_server_last_error(const pot3d_server *sv);

#ifdef __cplusplus
}
#endif
#endif /* POT3D_H */
