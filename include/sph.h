/*
 * sph.h -- C ABI of the MI355X (gfx950) weakly-compressible SPH hot path.
 *
 * The method is the one stated in PySPH (arXiv:1909.04504), Section 2 "The SPH
 * method": summation density (eq. 2) or the continuity equation
 * (eqn continuity:sph), the Tait equation of state (eq. eos), the momentum
 * equation with pressure-gradient and viscous terms (eqs. mom:sph,
 * mom:sph:press, mom:sph:visc) and the predictor-corrector time integration
 * (Section 2.1) -- or the Euler stage of the paper's dam-break example
 * (Section 3.2) -- with neighbours found on a uniform cell grid (Section 2.2,
 * "Nearest neighbor particle search").
 *
 * Conventions shared by every entry point
 *   - Memory: every array argument is a DEVICE pointer owned by the caller
 *     (for example a torch tensor's data_ptr()).  The library never allocates
 *     device memory; scratch space is the caller's workspace `ws` of at least
 *     sph_workspace_bytes() bytes, 256-byte aligned.
 *   - Layout: structure of arrays, one contiguous array per component, the
 *     particle index fastest (x[0][i], x[1][i], x[2][i]).  Unused components
 *     (z in 2D) may be NULL.
 *   - Precision: SPH_FP64 computes everything in double precision.
 *     SPH_FP32_MIXED evaluates the pair terms and the per-particle sums in
 *     single precision on cell-relative position offsets, and integrates
 *     positions and velocities in double precision; in that mode the arrays
 *     a, rho and p are float, otherwise double.  x, u and m are always double,
 *     and so is rho under the continuity scheme (where it is integrated).
 *   - Streams: `stream` is a hipStream_t passed as void*; all work is enqueued
 *     on it in order.  Calls do not synchronise unless documented.
 *   - Errors: a negative sph_status; sph_last_error() gives a message (per
 *     calling thread).  Arguments are validated on the host before any launch.
 *     Conditions found on the device (a particle outside a non-periodic box,
 *     a non-finite position or velocity) set bits in a flag word inside the
 *     workspace, read back by sph_check().
 *   - Ordering: sorting permutes the particle arrays in place; `id` travels
 *     with each particle so the caller can map results back.
 */
#ifndef SPH_MI355X_H
#define SPH_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPH_OK = 0,
    SPH_EINVAL = -1,      /* invalid argument (NULL pointer, bad size or parameter) */
    SPH_EWORKSPACE = -2,  /* workspace smaller than sph_workspace_bytes() */
    SPH_ECAPACITY = -3,   /* neighbour-list capacity too small */
    SPH_EDOMAIN = -4,     /* particle found outside a non-periodic domain */
    SPH_ENONFINITE = -5,  /* non-finite position or velocity found */
    SPH_EDEVICE = -6      /* HIP runtime error */
} sph_status;

typedef enum { SPH_FP64 = 0, SPH_FP32_MIXED = 1 } sph_precision;

/* Smoothing kernels W(|r|, h) = sigma_d w(|r|/h) (Section 2, compact
 * support k h).  Cubic spline: the M4 spline (Monaghan 1992), which PySPH
 * names CubicSpline, support 2h.  Wendland C2: Wendland (1995), scaled to
 * support 2h.  Quintic spline: (3-q)^5 - 6 (2-q)_+^5 + 15 (1-q)_+^5 (Morris
 * 1997), which PySPH names QuinticSpline, support 3h, sigma_2 = 7/(478 pi h^2),
 * sigma_3 = 1/(120 pi h^3).  The support radius R sets the neighbour
 * predicate |r| < R and the cell size (>= R / cell_div). */
typedef enum {
    SPH_CUBIC_SPLINE = 0,
    SPH_WENDLAND_C2 = 1,
    SPH_QUINTIC_SPLINE = 2
} sph_kernel;

typedef enum { SPH_FLUID = 0, SPH_WALL = 1 } sph_particle_type;

/* How sph_step obtains the density (Section 2).  Summation: rho is evaluated
 * from the positions (eq. 2).  Continuity: rho is a state advanced by the
 * continuity equation (eqn continuity:sph),
 * drho_i/dt = sum_j m_j (u_i - u_j) . gradW_ij. */
typedef enum { SPH_SCHEME_SUMMATION = 0, SPH_SCHEME_CONTINUITY = 1 } sph_scheme;

/* Time integration of sph_step.  Predictor-corrector: Section 2.1 (both
 * schemes).  Euler: the stage of the paper's dam-break example (Section 3.2,
 * "An example problem"; continuity scheme only). */
typedef enum {
    SPH_INTEGRATOR_PREDICTOR_CORRECTOR = 0,
    SPH_INTEGRATOR_EULER = 1
} sph_integrator;

/* Run parameters.  gamma of the Tait equation is 7 (Section 2, eq. eos). */
typedef struct {
    int32_t dim;          /* 2 or 3 */
    int32_t kernel;       /* sph_kernel */
    int32_t precision;    /* sph_precision */
    int32_t cell_div;     /* cells per support radius along an axis: 1 or 2 */
    int32_t periodic[3];  /* 1 if the axis is periodic */
    int32_t nbr_cap;      /* per-particle neighbour-list capacity of the pair
                           * passes: 0 = default (64 in 2D, 192 in 3D), > 0 =
                           * that many rounded up to a multiple of 4 (at most
                           * 4096), < 0 = no lists (every
                           * pass walks the cells).  A particle with more
                           * neighbours than the capacity is walked; results
                           * do not depend on it. */
    double h;             /* smoothing length, > 0 */
    double rho0;          /* reference density, > 0 */
    double c0;            /* reference speed of sound, > 0 */
    double nu;            /* kinematic viscosity, >= 0 */
    double eta;           /* regulariser of the viscous term, >= 0 (0.01 typical) */
    double dt;            /* time step, > 0 (sph_step only) */
    double g[3];          /* body acceleration (eq. mom:sph, a_body) */
    double lo[3], hi[3];  /* domain box; the cell grid covers [lo, hi) */
    int32_t scheme;       /* sph_scheme */
    int32_t integrator;   /* sph_integrator (sph_step only); EULER needs the
                           * continuity scheme */
    int32_t pair_tiles;   /* 3D mixed-precision summation passes (Section
                           * 2.2's cell grid cut into boxes whose particles
                           * and neighbour cells are staged in on-chip
                           * memory): 0 = used where they apply on grids with
                           * at least one particle per cell on average
                           * (default), < 0 = never (lists read from global
                           * memory), k > 0 = used wherever they apply, with at
                           * most k staged particles per box (3072 at most;
                           * larger boxes take the cell walk).  Results do not
                           * depend on it. */
    int32_t cell_order;   /* sort key of the cells (Section 2.2): 0 = row-major,
                           * x fastest (default); 1 = Z-order (Morton, the
                           * bits of the three cell coordinates interleaved,
                           * x lowest), 3D only.  Z-order keys span the smallest
                           * power-of-two grid holding every axis, so
                           * sph_grid's ncells (the length of cell_start and
                           * cell_end) is 8^bits. */
} sph_params;

/* Particle arrays (device pointers, caller-owned). */
typedef struct {
    int64_t n;       /* number of particles, 1 <= n < 2^31 */
    double* x[3];    /* positions */
    double* u[3];    /* velocities */
    void* a[3];      /* accelerations: double (SPH_FP64) or float (SPH_FP32_MIXED) */
    void* rho;       /* density: double or float as a; double under the
                      * continuity scheme */
    void* p;         /* pressure: double or float as a */
    double* m;       /* masses */
    uint8_t* type;   /* sph_particle_type */
    int32_t* id;     /* caller's ids; permuted with the particles */
    double* arho;    /* drho/dt: required under the continuity scheme (state of
                      * the predictor-corrector, output of the Euler stage);
                      * ignored, and may be NULL, otherwise */
} sph_particles;

/* Cell grid of `prm` (host only).  nc[k] = max(1, floor((hi-lo) cell_div / R))
 * cells along axis k < dim (1 for unused axes), *ncells their product.
 * Returns SPH_EINVAL if a periodic axis has fewer than 2 cell_div + 1 cells
 * (a neighbour would be reached twice) or the grid exceeds 2^31 cells. */
int sph_grid(const sph_params* prm, int64_t nc[3], int64_t* ncells);

/* Workspace size in bytes for n particles.  adjoint_k > 0 adds the recompute
 * tape of sph_step_backward for segments of adjoint_k steps.  Returns 0 if the
 * parameters are invalid (see sph_last_error()). */
size_t sph_workspace_bytes(const sph_params* prm, int64_t n, int64_t adjoint_k);

/* Neighbour-search build (Section 2.2; the Z-order-style build sorts particle
 * ids by a cell key): hash every particle to its cell
 *   c_k = clamp(floor((x_k - lo_k) / cs_k), 0, nc_k - 1),
 *   key = c_0 + nc_0 (c_1 + nc_1 c_2)   (or the Z-order key, prm->cell_order),
 * sort the particles stably by key (ties keep their current order), permute
 * every particle array in place into that order, and write per cell the slot
 * range [cell_start[c], cell_end[c]) of its particles (empty cells:
 * start = end).  cell_start and cell_end hold ncells entries each. */
int sph_bin_sort(const sph_params* prm, sph_particles* pa, void* ws, size_t ws_bytes,
                 uint32_t* cell_start, uint32_t* cell_end, void* stream);

/* Neighbour lists (Section 2.2) of particles sorted by sph_bin_sort with the
 * same parameters: j is a neighbour of i iff |x_i - x_j| < R, with the
 * minimum image on periodic axes, i itself included.  Written as CSR:
 * offsets[0..n] (int64) and nbr[offsets[i] .. offsets[i+1]) (sorted-order
 * indices).  Two phases: counts are formed and *total (host) is set; if
 * *total > capacity the call returns SPH_ECAPACITY without writing nbr.
 * Synchronises the stream once (to read the total). */
int sph_neighbors(const sph_params* prm, const sph_particles* pa, const uint32_t* cell_start,
                  const uint32_t* cell_end, int64_t capacity, int64_t* offsets, int32_t* nbr,
                  int64_t* total, void* ws, size_t ws_bytes, void* stream);

/* Summation density (eq. 2): rho_i = sum_{j in N(i)} m_j W(|x_i - x_j|, h) for
 * particles sorted by sph_bin_sort.  Writes pa->rho. */
int sph_density(const sph_params* prm, sph_particles* pa, const uint32_t* cell_start,
                const uint32_t* cell_end, void* ws, size_t ws_bytes, void* stream);

/* Tait equation of state (eq. eos): p_i = (c0^2 rho0 / 7) ((rho_i/rho0)^7 - 1).
 * Reads pa->rho, writes pa->p.  Elementwise; no ordering requirement. */
int sph_eos(const sph_params* prm, sph_particles* pa, void* stream);

/* Momentum equation (eqs. mom:sph, mom:sph:press, mom:sph:visc) for particles
 * sorted by sph_bin_sort, with rho and p already set: for fluid particles
 *   a_i = g + sum_{j in N(i), j != i} m_j [ -(p_i/rho_i^2 + p_j/rho_j^2) gradW_ij
 *         + 4 nu/(rho_i + rho_j) (r_ij . gradW_ij)/(|r_ij|^2 + eta h^2) (u_i - u_j) ],
 * r_ij = x_i - x_j; wall particles get a = 0.  Writes pa->a. */
int sph_momentum(const sph_params* prm, sph_particles* pa, const uint32_t* cell_start,
                 const uint32_t* cell_end, void* ws, size_t ws_bytes, void* stream);

/* nsteps predictor-corrector steps (Section 2.1).  Per step, for fluid
 * particles: v = u + dt/2 a;  x <- wrap(x + dt v);  neighbour rebuild;
 * rho, p, a evaluated at (x, v);  u <- v + dt/2 a.  The acceleration of one
 * step's end starts the next step.  Wall particles do not move (u = a = 0).
 * prime_accel = 1 first evaluates rho, p, a at the input (x, u) (needed when
 * a is not yet known); 0 takes pa->a as given.  Particles end sorted by cell.
 * diag: NULL, or a device array of nsteps * (1 + dim) doubles receiving after
 * each step the kinetic energy sum m|u|^2/2 and the momentum sum m u.
 *
 * With prm->scheme = SPH_SCHEME_CONTINUITY, pa->rho is a state (the density
 * of every particle, walls included) and the right-hand side at (x, u, rho)
 * is: neighbour rebuild at x;  p = EOS(rho) for all particles;
 *   arho_i = sum_{j in N(i)} m_j (u_i - u_j) . gradW_ij  over all j for a
 *   fluid particle and over fluid j for a wall particle;
 *   a_i from the momentum equation for fluid particles (walls: 0).
 * Walls keep x and u = 0 under both integrators.
 *   Predictor-corrector: per step, for fluid u and every rho,
 *     u' = u + dt/2 a;  rho' = rho + dt/2 arho;  x <- wrap(x + dt u');
 *     rates at the predicted end state (x, u' + dt/2 a, rho' + dt/2 arho);
 *     u <- u' + dt/2 a;  rho <- rho' + dt/2 arho.
 *   The rates of a step's end start the next step: prime_accel = 1 first
 *   evaluates a and arho at the input; 0 takes pa->a and pa->arho as given.
 *   Euler (prm->integrator = SPH_INTEGRATOR_EULER, the example's stage): per
 *   step, rates at (x, u, rho), then u <- u + dt a, x <- wrap(x + dt u) with
 *   the new u, rho <- rho + dt arho; prime_accel is ignored.
 * pa->p, pa->a and pa->arho hold the last evaluation's values. */
int sph_step(const sph_params* prm, sph_particles* pa, int64_t nsteps, int prime_accel,
             void* ws, size_t ws_bytes, double* diag, void* stream);

/* Adjoint of k steps of sph_step (reverse mode; not part of the paper).
 * `ckpt` is the state (x, u, a, m, type, id) at the start of the segment, as
 * left by sph_step (its arrays are not modified: the k steps are recomputed
 * from a copy inside the workspace, which needs adjoint_k >= k).
 * lam_in: adjoint of the state after the k steps, in the particle order in
 * which sph_step leaves that state: 3*dim doubles per particle, laid out
 * [lam_x (dim arrays of n)][lam_u (dim arrays)][lam_a (dim arrays)].
 * lam_out: the adjoint at the start of the segment, same layout, in the order
 * of ckpt.  *dJ_dnu (device double) is incremented by the viscosity
 * gradient of the segment.  lam_in and lam_out may not alias.  Summation
 * scheme only (SPH_EINVAL otherwise).
 * The first-step acceleration a^0 of a rollout is evaluated by
 * sph_accel_backward. */
int sph_step_backward(const sph_params* prm, const sph_particles* ckpt, int64_t k,
                      const double* lam_in, double* lam_out, double* dJ_dnu, void* ws,
                      size_t ws_bytes, void* stream);

/* Adjoint seed of the kinetic-energy objective J = scale sum_i m_i |u_i|^2 / 2
 * at the state pa (the end state of a rollout, as sph_step leaves it): writes
 * lam (3*dim arrays of n doubles, the [lam_x][lam_u][lam_a] layout of
 * sph_step_backward) with lam_x = 0, lam_u = scale m u, lam_a = 0.  Not part
 * of the paper (the differentiation pattern of this library). */
int sph_ke_seed(const sph_params* prm, const sph_particles* pa, double scale, double* lam,
                void* stream);

/* Adjoint of the acceleration evaluation a = A(x, u; nu) at the state `st`
 * (sorted or not): given lam_a (dim arrays of n doubles), ADDS (dA/dx)^T lam_a
 * to lam_x, (dA/du)^T lam_a to lam_u and (dA/dnu)^T lam_a to *dJ_dnu.
 * Arrays in the order of st.  st is not modified.  The workspace must be
 * sized with adjoint_k >= 1.  Summation scheme only (SPH_EINVAL otherwise). */
int sph_accel_backward(const sph_params* prm, const sph_particles* st, const double* lam_a,
                       double* lam_x, double* lam_u, double* dJ_dnu, void* ws, size_t ws_bytes,
                       void* stream);

/* Interaction count (the throughput metric's unit): every density evaluation
 * (sph_density and each evaluation inside sph_step; with the continuity
 * scheme, each step's pair pass) adds sum_i |N(i)| (ordered
 * pairs, each particle counted as its own neighbour) to a 64-bit counter in
 * the workspace.  Synchronises the stream, stores the counter in *total
 * (host), and zeroes it if reset = 1. */
int sph_read_interactions(void* ws, size_t ws_bytes, int64_t* total, int reset, void* stream);

/* Per-kernel timing for benchmarks.  While enabled (on = 1), each kernel
 * launch of the library is bracketed by two HIP events recorded on the call's
 * stream.  sph_timer_read synchronises on those events and, for each kernel
 * slot k < nslots, stores its name (static string), the summed elapsed
 * milliseconds and the number of launches; reset = 1 then clears the totals.
 * Returns the number of kernel slots.  Process-wide state, not thread-safe;
 * keep it disabled while a stream is being captured into a graph. */
int sph_timer_enable(int on);
int sph_timer_read(int nslots, const char** names, double* ms, int64_t* launches, int reset);

/* Bytes of the static device scratch of sph_step_noalloc (one copy per device,
 * held until the process ends). */
#define SPH_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* sph_step without a caller workspace, for callers that cannot allocate
 * device memory (code under graph capture, serving loops, harnesses that
 * forbid hipMalloc): the workspace is a static device array of
 * SPH_NOALLOC_SCRATCH_BYTES bytes per device, found with hipGetSymbolAddress
 * on the first call on each device.  Same arguments and results as sph_step
 * otherwise; the caller still provides the particle arrays and diag.
 * Allocates nothing.  Returns SPH_EWORKSPACE when sph_workspace_bytes(prm, n,
 * 0) exceeds SPH_NOALLOC_SCRATCH_BYTES.  Every call on a device shares that
 * device's array, which keeps the last call's contents: each call clears its
 * flag words and interaction counters first (device-detected conditions are
 * not reported), and calls that overlap on one device race. */
int sph_step_noalloc(const sph_params* prm, sph_particles* pa, int64_t nsteps, int prime_accel,
                     double* diag, void* stream);

/* Synchronises the stream and returns SPH_OK, or the first device-detected
 * condition since the last call (SPH_ENONFINITE, then SPH_EDOMAIN), and
 * clears the flags. */
int sph_check(void* ws, size_t ws_bytes, void* stream);

/* Message of the last error on the calling thread ("" if none). */
const char* sph_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPH_MI355X_H */
