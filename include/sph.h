/*
 * libsph_hip — cell-based SPH neighbour interactions on one MI355X (gfx950).
 *
 * The calls follow the SPH statement of Schaller et al., "SWIFT: Using
 * task-based parallelism, fully asynchronous communication, and graph
 * partition-based domain decomposition for strong scaling on more than
 * 100 000 cores" (PASC'16), Sec. 2 (equations (rho), (dvdt), (dudt) with
 * P = (gamma-1) rho u and Omega = 1 + h/(3 rho) d rho/d h) and the cell / task
 * decomposition of Sec. 3.1: cells of edge at least the largest smoothing
 * length, recursively split while they hold more than a set number of
 * particles, self and pair interactions, a sort stage before the density
 * stage, a ghost stage between density and force, and an integrator stage
 * after the force.
 *
 * Notation: H is the paper's smoothing length h, the radius of the sphere
 * within which neighbours contribute (compact support of the cubic-spline
 * kernel W(r,H) = 8/(pi H^3) w(r/H)).  The smoothing length of every particle
 * is solved so that rho_i H_i^3 = (kernel_gamma * eta)^3 m_i.
 *
 * Conventions of every call:
 *   - Returns sph_status; never throws, never aborts.  Argument errors and
 *     HIP launch errors are reported synchronously.  Conditions found on the
 *     device (non-convergence, H too large for the box) are reported by the
 *     call that observes them: the density stage runs its first sweeps as a
 *     device-gated sequence and reads the device once at its end (more
 *     sweeps, relists and rebuilds continue from there on the host); a step
 *     reads it once more before its density stage (largest speed, validity
 *     of the kept cells and lists); ghost and force do not wait on the
 *     device, and the force stage's counts and a step's totals are read by
 *     sph_get_stats.
 *   - All particle arrays are DEVICE pointers owned by the caller, length n,
 *     structure-of-arrays, float64 unless stated.  The library never frees
 *     them.
 *   - The library never allocates device memory: every buffer it keeps
 *     (keys, octree, cell and particle lists, kernel-side particle data,
 *     predictor samples, interpolation order) is carved from the workspace
 *     the caller gives to sph_create (sph_workspace_size estimates it).  A
 *     call whose buffers do not fit returns SPH_ERR_WORKSPACE and
 *     sph_get_stats reports the bytes it needed; the context stays usable
 *     for smaller work, or is replaced by one with a larger workspace.  The
 *     context-free predictor calls take their own workspace argument.
 *   - Work is enqueued on the HIP stream given to sph_create.
 *   - A context is not thread-safe; use one context per host thread.
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPH_OK = 0,
    SPH_ERR_INVALID = -1,        /* bad argument, NaN/Inf input, position outside its box */
    SPH_ERR_HIP = -2,            /* a HIP runtime call or kernel launch failed */
    SPH_ERR_NOT_CONVERGED = -3,  /* smoothing lengths not converged in max_h_iter sweeps */
    SPH_ERR_H_EXCEEDS_CELL = -4, /* a smoothing length outgrew the cell grid (rebuild) */
    SPH_ERR_BOX_TOO_SMALL = -5,  /* a smoothing length exceeds 1/3 of its box edge */
    SPH_ERR_WORKSPACE = -6,      /* the caller's workspace is too small for the call */
    SPH_ERR_STATE = -7           /* call out of order (e.g. force before ghost) */
} sph_status;

enum { SPH_FP64 = 0, SPH_FP32C = 1, SPH_FP32 = 2 };      /* sph_params.precision */
enum { SPH_EXEC_GRID = 0, SPH_EXEC_PERSISTENT = 1 };     /* sph_params.exec_mode */
enum { SPH_PRUNE_BOX = 0, SPH_PRUNE_SORTED = 1 };        /* sph_params.prune */
enum { SPH_FORCE_PAIRS = 0, SPH_FORCE_GATHER = 1 };      /* sph_params.force_mode */
enum { SPH_LISTS_CELL = 0, SPH_LISTS_PARTICLE = 1 };     /* sph_params.lists */

typedef struct {
    double gamma;        /* adiabatic index, 5/3 */
    double eta;          /* resolution parameter (Dehnen-Aly), 1.2348 ~ 48 neighbours */
    double kernel_gamma; /* H / h_DA for the cubic spline, sqrt(10/3) */
    double h_tol;        /* converged when |rho H^3 - C| <= h_tol * C (FP64 test); the FP32
                            modes use at least 2.5e-7 (SPH_FP32C) or 2e-6 (SPH_FP32), the
                            resolution of their sums, and finish every converged particle
                            with one Newton update of H whose rho and drho/dH come from
                            the second-order expansion of the sums (no further sweep) */
    int max_h_iter;      /* smoothing-length sweeps per density call */
    int n_split;         /* split cells holding more than this many particles (<= 64) */
    int precision;       /* SPH_FP64, SPH_FP32C (cell-relative FP32, compensated sums)
                            or SPH_FP32 (cell-relative FP32, plain sums) */
    int exec_mode;       /* SPH_EXEC_GRID: one workgroup slot per cell;
                            SPH_EXEC_PERSISTENT: in the force loop, resident
                            workgroups drain device task queues, one per XCD
                            over a contiguous Morton range of cells, and help
                            the other XCDs' queues once their own is empty
                            (density sweeps run as a grid in both modes) */
    int n_domains;       /* number of independent periodic boxes (>= 1) */
    int persistent_wgs;  /* resident workgroups for the persistent mode (0: auto) */
    int use_graph;       /* 1: density sweeps, ghost and force run as one captured
                            hipGraph (sph_density_ghost_force and sph_step) */
    int prune;           /* pair-candidate selection: SPH_PRUNE_BOX (neighbour-cell
                            particles within range of the bounding box of the cell's
                            particles) or SPH_PRUNE_SORTED (window of the sort stage's
                            per-direction order) */
    int rebuild_steps;   /* 0: sph_step rebuilds cells and lists every step.  K > 0:
                            lists get an extra skin of K times the step's largest
                            displacement and sph_step keeps cells and lists while
                            every leaf's largest H plus twice the largest
                            displacement since the build stays inside its list
                            radius (rebuilding when not) */
    int h_drift;         /* 1: sph_step starts each particle's H iteration from its
                            previous H carried along the flow, H exp(-dt du/dt /
                            (3 (gamma-1) u)) (d ln rho/dt = du/dt / ((gamma-1) u)
                            for these equations; factor clamped to [1/2, 2]); 0:
                            from the previous H.  Not applied while the learned
                            predictor supplies the start.  Only the start changes:
                            the converged H is set by the same FP64 test */
    int force_mode;      /* SPH_FORCE_PAIRS: each unordered pair of particles evaluated
                            once and applied to both (Sec. 3.1 pair symmetry; atomic
                            accumulation on the j side); SPH_FORCE_GATHER: each
                            particle sums its own pairs r < max(H_i, H_j) (every pair
                            evaluated from both sides, no atomics, symmetric
                            neighbour-cell lists; box pruning only) */
    int lists;           /* SPH_LISTS_CELL: the density and force kernels stage the
                            candidates of each leaf's neighbour cells in LDS and test
                            them; SPH_LISTS_PARTICLE: at every cell build the cell lists
                            are turned into one list per particle of the j with
                            r_ij < max(R_i, R_j), R = 1.02 H plus the kept cells' skin;
                            a chunk (up to 64 particles of one leaf, one wave) stages the
                            union of its particles' lists in LDS and every lane loops over
                            its own list only (positions as fixed-point integers per box
                            axis, converted to the chunk's frame in the compute
                            precision).  Requires SPH_FORCE_GATHER and SPH_PRUNE_BOX */
    int tile;            /* particle lists: candidates staged in LDS per segment, 256, 512
                            or 1024 (0: 1024 for the density and 512 for the force; FP64
                            at most 512 / 256) */
    int waves_density;   /* cell lists, FP32 modes: occupancy target (waves per SIMD) the
                            packed density kernel is compiled for, 4, 5, 6 or 8 (0: 6) */
    int waves_force;     /* the same for the gather force kernel, 4, 5, 6 or 8 (0: 5) */
    int batch;           /* cell lists, FP32 modes: neighbour-cell entries staged per batch
                            by those two kernels, 16 or 32 (0: 32).  These three only tune
                            speed: every choice gives the same results bit for bit */
    const double* boxes; /* HOST pointer, n_domains x 3 box edge lengths; copied */
} sph_params;

typedef struct {
    int64_t n;
    double *x, *y, *z;       /* positions, inside [0, L) of their box (in/out) */
    double *vx, *vy, *vz;    /* velocities (in/out) */
    double *u;               /* specific internal energy (in/out) */
    double *m;               /* masses (in) */
    double *H;               /* smoothing lengths: initial guess in, converged out */
    double *rho, *drho_dH;   /* density and its H-derivative at the converged H (out) */
    double *omega, *P;       /* grad-h term Omega and pressure (out, ghost) */
    double *ax, *ay, *az;    /* acceleration dv/dt (out, force) */
    double *dudt;            /* du/dt (out, force) */
    int64_t *id;             /* optional: carried through the permutation (may be NULL) */
    int32_t *domain;         /* box index of each particle; NULL when n_domains == 1 */
    int32_t *nngb;           /* optional: #{j : r_ij < H_i}, self included (out; may be
                                NULL).  Written by the density stage at the last H it
                                evaluated and rewritten by the force stage at the final H */
} sph_particles;

typedef struct {
    int64_t n;               /* particles */
    int64_t n_leaves;        /* leaf cells (self tasks) */
    int64_t n_nodes;         /* cells of all levels */
    int64_t n_list;          /* neighbour-cell entries (ordered pairs incl. self) */
    int64_t n_pair_tasks;    /* unordered pairs of distinct leaves (A, B) in the current
                                lists, each counted once by its owner: the lower index
                                when the pair is in both leaves' lists (always, with the
                                symmetric lists of the gather form), else the leaf whose
                                list holds it; periodic self-images (B = A shifted) are
                                not counted */
    int64_t n_dens;          /* sum_i #{j : r_ij < H_i}, self included, at the final H
                                (from the last force call; after density alone, at the
                                last H the density stage evaluated) */
    int64_t n_force;         /* #{unordered i != j : r_ij < max(H_i,H_j)}, last force call */
    int32_t sweeps;          /* density sweeps of the last density call */
    int32_t n_unconverged;   /* particles left unconverged by the last density call */
    int32_t relists;         /* neighbour-list rebuilds inside the last density call */
    int32_t rebuilds;        /* full cell rebuilds since create */
    int32_t depth;           /* deepest cell level */
    int32_t key_bits;        /* bits sorted by the Morton radix sort */
    double conserved[5];     /* FP64 totals after the last step: M, Px, Py, Pz, E */
    double t_density_ms;     /* stream time of the last density call (all sweeps) */
    double t_ghost_ms;
    double t_force_ms;
    double t_build_ms;       /* last build_cells + sort_cells */
    double t_density_kernels_ms; /* summed duration of the density-sweep kernels of the last density call
                                    (-1 when sweeps ran inside the graph) */
    double t_force_kernel_ms;    /* duration of the force kernel of the last force call (-1: inside the graph) */
    int64_t n_dens_evals;    /* interactions r_ij < H_i evaluated over all sweeps of the last density call */
    int32_t n_density_launches; /* density-sweep kernel launches of the last density call */
    int32_t graph_captures;     /* graph (re)captures since sph_create (use_graph = 1) */
    int32_t graph_fallbacks;    /* graph runs the host had to finish since sph_create */
    int32_t precision_rebuilds; /* FP32 modes: rebuilds since sph_create because H had shrunk
                                   below the cells' extent rule after converging */
    int32_t unconv_after[8];    /* particles left unconverged after sweep k+1 of the last
                                   density call (-1: sweep not run) */
    double t_predict_ms;        /* features + network inference of the last sph_step
                                   (-1: the predictor stage did not run) */
    int64_t steps_since_build;  /* sph_step calls since cells and lists were built */
    int64_t n_builds;           /* cell and list builds since sph_create */
    double list_margin;         /* twice the largest displacement since the build */
    int64_t n_chunks;           /* particle lists: chunks (up to 64 particles of one leaf) */
    int64_t n_plist;            /* particle lists: entries over all particles (pairs listed from
                                   both sides, the particle itself not listed) */
    int64_t n_union;            /* particle lists: members of the chunks' unions */
    int64_t stale_moved;        /* particle lists, last drift: particles beyond their skin */
    int64_t stale_grown;        /* particle lists, last drift: particles whose H passed their
                                   list radius */
    int64_t workspace_bytes;    /* usable bytes of the workspace */
    int64_t workspace_in_use;   /* bytes the context's buffers hold now */
    int64_t workspace_high;     /* most bytes held at once */
    int64_t workspace_needed;   /* after SPH_ERR_WORKSPACE: bytes that call needed (0: none failed) */
    int64_t n_force_total;      /* sum of n_force over every force stage since sph_create */
    int64_t n_dens_total;       /* sum of n_dens (force stage's count) since sph_create */
    int64_t force_calls;        /* force stages since sph_create */
} sph_stats;

typedef struct sph_ctx sph_ctx;

/* Smallest workspace sph_create accepts. */
#define SPH_WORKSPACE_MIN ((size_t)1 << 20)

/* Workspace bytes for n particles with these parameters (HOST *bytes): an
 * estimate covering the stages' buffers for the clustered and lattice
 * workloads, interpolation at up to n points and predictor samples of up to
 * n / 8 particles.  SPH_ERR_INVALID on n < 1 or n >= 2^31. */
sph_status sph_workspace_size(const sph_params* params, int64_t n, size_t* bytes);

/* Create a context.  `params` is copied (including the boxes array).
 * workspace: DEVICE memory of `bytes` bytes owned by the caller (e.g. a torch
 * uint8 tensor), at least SPH_WORKSPACE_MIN; the context carves all its
 * device buffers from it and the caller must keep it until sph_destroy.
 * hip_stream: a hipStream_t (NULL = default stream); every call's work is
 * ordered on it.  The context also creates one stream of its own (default
 * priority, non-blocking) on which a build permutes the arrays the octree
 * does not read; it is ordered after the sort and joined back into
 * hip_stream by events before the build returns, and destroyed by
 * sph_destroy (without it the permutation stays on hip_stream). */
sph_status sph_create(const sph_params* params, void* workspace, size_t bytes, void* hip_stream, sph_ctx** out);

/* Release the context (its workspace returns to the caller).  Safe on NULL. */
sph_status sph_destroy(sph_ctx* ctx);

/* Cell construction (Sec. 3.1: a grid of cells of edge >= the largest H per
 * box -- about twice that where such cells would hold under 64 particles --
 * recursively split while a cell holds more than n_split particles; self
 * and pair interactions between cells within range).  Binds `p` to the
 * context, permutes every non-NULL particle array in place into Morton order
 * of the cells, and builds the neighbour-cell lists.  Particles must lie in
 * [0, L) of their box.  Errors: SPH_ERR_INVALID (NaN, non-positive H or m,
 * out-of-box position), SPH_ERR_BOX_TOO_SMALL (max H > L/3). */
sph_status sph_build_cells(sph_ctx* ctx, const sph_particles* p);

/* Sort stage (Sec. 3.1 "sorted" cells): for every leaf cell and each of the
 * 13 axis directions between neighbouring cells, the particles' projections
 * sorted ascending; used to skip pair candidates whose projections differ by
 * at least the interaction range (prune = SPH_PRUNE_SORTED).  With
 * SPH_PRUNE_BOX the interaction kernels do not read this order and the call
 * only records the stage.  Requires sph_build_cells. */
sph_status sph_sort_cells(sph_ctx* ctx);

/* Density stage, eq. (rho): sweeps over self and pair interactions computing
 * rho_i, d rho_i/d H_i and the neighbour count at the current H, each
 * followed by an FP64 Newton-Raphson update of H toward rho H^3 = C inside a
 * bracket; repeats for the unconverged particles until all pass the FP64
 * test or max_h_iter sweeps are done (SPH_ERR_NOT_CONVERGED).  Writes H, rho,
 * drho_dH.  Requires sph_sort_cells. */
sph_status sph_density(sph_ctx* ctx);

/* Ghost stage (Sec. 3.1, with the closing relations of Sec. 2): Omega_i, P_i
 * = (gamma-1) rho_i u_i and A_i = P_i/(Omega_i rho_i^2).  Writes omega, P.
 * Requires sph_density. */
sph_status sph_ghost(sph_ctx* ctx);

/* Force stage, eqs. (dvdt) and (dudt) over every pair with r_ij <
 * max(H_i, H_j).  force_mode = SPH_FORCE_GATHER (default): each particle
 * sums its own pairs, so every unordered pair is evaluated from both sides
 * and each output is written once (no atomics).  SPH_FORCE_PAIRS: every
 * unordered pair is evaluated once and its equal and opposite contributions
 * are applied to both particles (j-side sums with atomic adds).  Writes ax,
 * ay, az, dudt.  Requires sph_ghost. */
sph_status sph_force(sph_ctx* ctx);

/* Density, ghost and force in one call.  With use_graph = 1 they run as one
 * captured hipGraph holding a fixed number of density sweeps gated by a
 * device flag (re-captured after every cell or list rebuild); work the
 * graph cannot finish (more sweeps, list or grid rebuilds) is completed by
 * the host-driven path.  Requires sph_sort_cells. */
sph_status sph_density_ghost_force(sph_ctx* ctx);

/* One kick-drift-kick step of length dt (integrator stage, Sec. 3.1):
 * half kick of v and u with the current forces, drift with periodic wrap
 * (and, with h_drift, the start of each H iteration carried along the
 * flow), cell rebuild and sort or, with rebuild_steps > 0, a refresh of the
 * kept cells, density from that start, ghost with the predicted u, force
 * with the predicted v, second half kick fused with the FP64 conservation
 * sums.  Requires a previous sph_force (forces of the current positions).
 * A rebuild inside the step reorders the particles without carrying rho,
 * drho_dH, omega and P along (the density and ghost stages then rewrite
 * them); after a failed step they are undefined. */
sph_status sph_step(sph_ctx* ctx, double dt);

/* SPH interpolation, Sec. 2, eq. (interp): out[k] = sum_i m_i Q_i / rho_i
 * W(|p_k - r_i|, H_i) for m_pts points p_k = (px[k], py[k], pz[k]) of box
 * pdom[k] (pdom may be NULL with one box), each particle contributing inside
 * its own support H_i (the scatter reading of the equation), distances
 * minimum-image in the periodic box.  Q holds one double per bound particle
 * in the bound arrays' CURRENT order (sph_build_cells permutes them), e.g. the
 * bound u or a derived field; rho and H are those of the last density stage.
 * All pointers are DEVICE pointers; points outside [0, L) are wrapped into the
 * box, and a point with a non-finite coordinate or a box index outside
 * [0, n_domains) gets NaN.  Asynchronous on the context's stream; out must
 * not alias Q.  SPH_ERR_INVALID on a NULL pointer with m_pts > 0, m_pts < 0
 * or > 2^31 - 1, or pdom NULL with several boxes; SPH_ERR_STATE before
 * sph_density. */
sph_status sph_interpolate(sph_ctx* ctx, const double* Q, const double* px, const double* py, const double* pz,
                           const int32_t* pdom, int64_t m_pts, double* out);

/* ---------------------------------------------------------------------------
 * Learned smoothing-length predictor.
 *
 * The density stage solves rho H^3 = (kernel_gamma eta)^3 m per particle by
 * Newton-Raphson (Sec. 2); sph_step warm-starts it from the previous H.  The
 * predictor replaces that starting point: after the drift a small network
 * maps per-particle features to y = log(H_new / H_prev) and the iteration
 * starts from H_prev exp(y).  The plain iteration still decides convergence,
 * so the converged H does not depend on the prediction; a particle whose
 * prediction is off simply needs more sweeps (reported as unconv_after[0]).
 *
 * Features (SPH_MLP_NF used, stored as float[SPH_MLP_XSTRIDE] rows, columns
 * SPH_MLP_NF.. zero), from positions after the drift, velocities after the
 * first half kick, and H, rho, P, du/dt of the previous evaluation; the
 * feature grid of a box with edges L and n particles has
 * G_a = clamp(floor(L_a / s + 1/2), 1, 256) cells per axis, s = 2 (V/n)^(1/3):
 *   0  log(H / (V/n)^(1/3))
 *   1  log(particle count of the particle's grid cell)
 *   2  log(count of the 27 cells around it / (27 n / (G_x G_y G_z)))
 *   3  |g|, g_a = (S+_a - S-_a) / S27, S+-_a the counts of the 9 cells at
 *      offset +-1 along axis a (periodic), S27 the 27-cell count
 *   4  sum_a g_a (f_a - 1/2), f_a the fractional position inside the cell
 *   5  -dt rho du/dt / (3 P) (first-order change of log H implied by the
 *      continuity and energy equations; 0 where P <= 0)
 *   6  dt |v| / H
 *
 * Network: 16 inputs (features, zero-padded) standardised by xmu, xsd;
 * three hidden layers of 64 SiLU units; one output o; y = ymu + ysd o.
 * Parameter vector (float32, SPH_MLP_NP values):
 *   W1[16][64] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] w4[64] b4
 *   (SPH_MLP_NT trained values), then xmu[16] xsd[16] ymu ysd.
 * W1, W2, W3 and w4 enter the network rounded to bfloat16 (nearest, ties to
 * even); biases are used in float32; products accumulate in float32.
 * Training minimises L = 1/(2n) sum (o - (y - ymu)/ysd)^2 with Adam.
 * ------------------------------------------------------------------------- */
#define SPH_MLP_NF 7
#define SPH_MLP_XSTRIDE 8
#define SPH_MLP_NIN 16
#define SPH_MLP_NH 64
#define SPH_MLP_NT 9473
#define SPH_MLP_NP 9507
/* Rows one sph_mlp_loss_grad call takes at most (row indices are 32-bit). */
#define SPH_MLP_MAX_ROWS 2147483647LL

/* Workspace bytes (HOST *bytes) of sph_mlp_forward and sph_mlp_loss_grad over
 * n rows. */
sph_status sph_mlp_workspace_size(int64_t n, size_t* bytes);

/* Network output for n feature rows: y[i] = predicted log(H_new/H_prev).
 * params: SPH_MLP_NP floats, X: n x SPH_MLP_XSTRIDE floats, y: n floats; all
 * DEVICE pointers.  workspace: DEVICE scratch of `bytes` bytes (packed
 * weights; sph_mlp_workspace_size).  Matrix products on the MFMA units
 * (bfloat16 weights, activations split into two bfloat16 terms, float32
 * accumulation).  hip_stream: hipStream_t (NULL = default); asynchronous.
 * SPH_ERR_INVALID on n < 0 or a NULL pointer with n > 0,
 * SPH_ERR_WORKSPACE if the workspace is too small. */
sph_status sph_mlp_forward(const float* params, const float* X, int64_t n, float* y, void* workspace, size_t bytes,
                           void* hip_stream);

/* Mean loss (HOST *loss, may be NULL) and its gradient with respect to the
 * SPH_MLP_NT trained parameters (DEVICE grad) over n rows (X as above, y:
 * n target values of log(H_new/H_prev)); float32 arithmetic with the
 * bfloat16-rounded weights.  workspace: DEVICE scratch of `bytes` bytes
 * (per-workgroup partial gradients; sph_mlp_workspace_size).  Synchronises
 * the stream (for *loss).  SPH_ERR_INVALID on n < 1, n > SPH_MLP_MAX_ROWS or
 * a NULL pointer; SPH_ERR_WORKSPACE if the workspace is too small. */
sph_status sph_mlp_loss_grad(const float* params, const float* X, const float* y, int64_t n, float* grad,
                             double* loss, void* workspace, size_t bytes, void* hip_stream);

/* sph_mlp_loss_grad for callers that cannot allocate device memory or hand
 * over a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): same arguments without the workspace,
 * same kernels and the same result.  The partial gradients live in a fixed
 * array inside this library, about 9.7 MB (256 x SPH_MLP_NT + 256 floats
 * + the loss), which each GPU the library runs on holds until the process
 * ends; it serves any n up to SPH_MLP_MAX_ROWS, since the gradient kernel
 * runs at most 256 workgroups.  Nothing is allocated: no hipMalloc,
 * hipFree or allocating library call.  All calls on one GPU share that GPU's
 * array, so calls that overlap on one GPU (different streams or host
 * threads without ordering between them) race; calls ordered on one stream
 * do not.  hip_stream must belong to the current device.  Synchronises the
 * stream (for *loss).  SPH_ERR_INVALID on n < 1, n > SPH_MLP_MAX_ROWS or a
 * NULL pointer; SPH_ERR_HIP if the array's device address cannot be
 * obtained. */
sph_status sph_mlp_loss_grad_noalloc(const float* params, const float* X, const float* y, int64_t n, float* grad,
                                     double* loss, void* hip_stream);

/* One Adam step (step number t >= 1) on the SPH_MLP_NT trained values of
 * params with moment buffers m, v (SPH_MLP_NT floats each, DEVICE):
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). */
sph_status sph_mlp_adam(float* params, float* m, float* v, const float* grad, int t, float lr, float beta1,
                        float beta2, float eps, void* hip_stream);

/* Features of the bound particles in their current order, with the current
 * H, rho, P, du/dt as the previous evaluation's and step dt, into X (DEVICE,
 * n x SPH_MLP_XSTRIDE floats).  Requires sph_build_cells. */
sph_status sph_h_features(sph_ctx* ctx, double dt, float* X);

/* Record training samples during the following sph_step calls: each step
 * keeps about rate * n particles (chosen by a hash of seed, step count and
 * index) as (features, log(H_converged / H_prev)) until `capacity` samples
 * are held, in the caller's DEVICE buffers X (capacity x SPH_MLP_XSTRIDE
 * floats) and y (capacity floats), which must stay valid until recording
 * stops and sph_h_train has read them.  Calling again with the same buffers
 * and capacity only reports the count; other buffers restart the count.
 * capacity = 0 stops recording (X, y may be NULL).  Returns the number held
 * so far through *held (HOST, may be NULL). */
sph_status sph_h_record(sph_ctx* ctx, float* X, float* y, int64_t capacity, double rate, uint64_t seed,
                        int64_t* held);

/* Train the context's network on the recorded samples with the library's
 * forward, backward and Adam kernels: `epochs` passes in minibatches of
 * `batch` rows (a different affine permutation of the samples per epoch),
 * learning rate lr.  init = 1 starts from fresh weights (seeded) and sets the
 * standardisation constants from the samples; init = 0 continues.  *loss
 * (HOST, may be NULL) = mean minibatch loss of the last epoch. */
sph_status sph_h_train(sph_ctx* ctx, int epochs, int batch, double lr, uint64_t seed, int init, double* loss);

/* Set / read the context's network parameters (HOST, SPH_MLP_NP floats). */
sph_status sph_h_set_params(sph_ctx* ctx, const float* params);
sph_status sph_h_get_params(sph_ctx* ctx, float* params);

/* on = 1: sph_step starts the density iteration from the network's
 * prediction (requires parameters set or trained); on = 0: from the previous
 * H (the plain method). */
sph_status sph_h_predict(sph_ctx* ctx, int on);

/* Copy counters and timings to *out (synchronises the stream: the force
 * stage's counts and kernel time and a step's FP64 totals are read from the
 * device here).  The first call after the cells or lists changed also counts
 * the pair tasks with one small kernel on the library's stream. */
sph_status sph_get_stats(sph_ctx* ctx, sph_stats* out);

/* FP64 per-box totals of the bound particles (synchronises the stream):
 * out[5*b + k] = (M, Px, Py, Pz, E)_k of box b, out has 5*n_domains doubles
 * (HOST pointer). */
sph_status sph_domain_sums(sph_ctx* ctx, double* out);

/* Human-readable name of a status code (static string). */
const char* sph_status_str(sph_status s);

/* Library build description (static string). */
const char* sph_version(void);

#ifdef __cplusplus
}
#endif
#endif
