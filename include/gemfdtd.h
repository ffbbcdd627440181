/*
 * gemfdtd.h -- C ABI of the MI355X FDTD library.
 *
 * The library advances Maxwell's equations on a Yee grid with the leapfrog
 * scheme of the paper (Sec. III-B, Eq. 7-9): per time step an H layer
 * gathers curl-E messages into the magnetic nodes, then an E layer gathers
 * curl-H messages into the electric nodes, with fixed per-node weights
 * (Prop. 1 and Prop. 2, Sec. IV-A).  The regular Yee graph is kept implicit:
 * the edge weights are folded into per-cell coefficients.  A second
 * constructor builds the explicit graph (compressed sparse rows) and runs
 * the same two layers as generic weighted gathers.  The outer boundary is a
 * convolutional PML (CPML) backed by PEC; the paper's own absorbing layer
 * is the split-field PML of Sec. III-C, which this library replaces.
 *
 * Conventions (all calls):
 *  - ndim == 2 is the TMz polarisation (Ez, Hx, Hy), the paper's 2D
 *    polarisation of Eq. 3-5 up to the relabelling Ez = -Ey, Hy = Hz.
 *    ndim == 3 is the six-component Yee scheme.
 *  - Grid arrays are row-major with the last axis contiguous:
 *    2D idx = i*ny + j; 3D idx = (i*ny + j)*nz + k.  Sizes count CPML cells.
 *  - Cell (i,j[,k]) owns Ez(i,j) [3D: Ex(i+1/2,j,k), Ey(i,j+1/2,k),
 *    Ez(i,j,k+1/2)] and Hx(i,j+1/2), Hy(i+1/2,j) [3D: Hx(i,j+1/2,k+1/2),
 *    Hy(i+1/2,j,k+1/2), Hz(i+1/2,j+1/2,k)].  Its eps_r and sigma apply to its
 *    E components, its mu_r to its H components.
 *  - Outer boundary PEC: E components tangential to the planes i=0, j=0
 *    (k=0) are never updated; values beyond the last cell read as zero.
 *  - One step n -> n+1: H layer (H^{n+1/2}), E layer (E^{n+1}), soft source
 *    E[src] += amp*g((n+1) dt), probe sample index n = E^{n+1} at the probe.
 *  - Fields, coefficients and auxiliary CPML values are float32 on the
 *    device.  Coefficients are computed in double on the host and rounded
 *    once.
 *  - Device pointers are HIP device addresses on the device that was
 *    current when the handle was created.  Host pointers are ordinary
 *    memory.  Every call returns 0 (FDTD_OK) or a negative status; no call
 *    aborts or throws.  fdtd_last_error() gives a message for the calling
 *    thread's last failure.
 *  - A handle is used by one thread at a time.  Work is enqueued on the
 *    handle's stream; calls that return host data synchronise that stream.
 */
#ifndef GEMFDTD_H
#define GEMFDTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FDTD_OK = 0,
    FDTD_EINVAL = -1,      /* invalid argument */
    FDTD_EUNSTABLE = -2,   /* dt above the Courant limit c0 dt <= 1/sqrt(sum 1/d^2) */
    FDTD_ENOMEM = -3,      /* device allocation failed */
    FDTD_EDEVICE = -4,     /* a HIP call failed */
    FDTD_ENONFINITE = -5,  /* a field holds NaN or Inf */
    FDTD_ESTATE = -6       /* call not valid in the handle's current state */
};

/* Field components. */
enum { FDTD_EX = 0, FDTD_EY = 1, FDTD_EZ = 2, FDTD_HX = 3, FDTD_HY = 4, FDTD_HZ = 5 };

/* Source waveforms g(t) (the paper names Gaussian, sinusoidal and
 * modulated Gaussian sources, Sec. V-A and V-B, without formulas; these are
 * the forms used here).  The field gets amp * g(t):
 *  GAUSSIAN params {amp, t0, tau}: g = exp(-((t - t0)/tau)^2)
 *  RICKER   params {amp, t0, f}:   g = (1 - 2a) exp(-a), a = (pi f (t - t0))^2
 *  TABLE    g[n] given for the steps 0..n_table-1 (sample n is added at the
 *           end of step n, i.e. at time (n+1) dt), zero afterwards; amp = 1.
 *  SINE     params {amp, f, t_ramp}: g = r(t) sin(2 pi f t), with the
 *           turn-on r = sin^2(pi t / (2 t_ramp)) for t < t_ramp, else 1
 *           (t_ramp = 0: no ramp)
 *  MODGAUSS params {amp, t0, tau, f}: g = exp(-((t - t0)/tau)^2)
 *           sin(2 pi f (t - t0)) (four parameters) */
enum { FDTD_SRC_GAUSSIAN = 0, FDTD_SRC_RICKER = 1, FDTD_SRC_TABLE = 2, FDTD_SRC_SINE = 3, FDTD_SRC_MODGAUSS = 4 };

/* Optional device allocator.  alloc returns NULL on failure.  The library
 * frees every block it allocated in fdtd_destroy / fdtd_batch_destroy. */
typedef struct {
    void *ctx;
    void *(*alloc)(void *ctx, size_t bytes, void *stream);
    void (*free)(void *ctx, void *ptr, void *stream);
} fdtd_allocator;

/* CPML profile (the paper gives no absorbing-layer constants).  For an axis
 * with d cells at a face, normalised depth rho = distance into the layer / d
 * (1 at the PEC wall), sampled at x = i for E-type and x = i + 1/2 for
 * H-type differences:
 *   sigma = sigma_max rho^m, kappa = 1 + (kappa_max - 1) rho^m,
 *   alpha = alpha_max (1 - rho)^m_alpha,
 *   b = exp(-(sigma/kappa + alpha) dt/eps0),
 *   c = sigma (b - 1)/(kappa (sigma + kappa alpha)).
 * sigma_max <= 0 selects 0.8 (m + 1)/(eta0 d_axis).  kappa_max < 1 is
 * invalid.  npml faces: -x, +x, -y, +y, -z, +z. */
typedef struct {
    int32_t npml[6];
    double m, sigma_max, kappa_max, alpha_max, m_alpha;
    /* 0: the CPML above.  1 (ndim 2 only): the paper's split-field PML
     * (Sec. III-C, Eq. 10-13 in TMz form): in the layer cells Ez = Ezx +
     * Ezy with eps dEzx/dt + sigma_x Ezx = dHy/dx, eps dEzy/dt + sigma_y Ezy
     * = -dHx/dy, and mu dHx/dt + sm_y Hx = -dEz/dy, mu dHy/dt + sm_x Hy =
     * dEz/dx, with the magnetic conductivity sm matched (sm / mu0 = sigma /
     * eps0), sigma graded as above (kappa_max and alpha_max unused),
     * discretised with the semi-implicit averaging of Eq. 7-9.  The layer
     * cells must be vacuum (eps_r = mu_r = 1, sigma = 0).  Kernel variant 1
     * and the explicit graph (4 nodes per cell) only. */
    int32_t split;
} fdtd_cpml;

/* Problem description (the paper's problem statement, Sec. III: grid and
 * steps, per-cell eps, mu, sigma, absorbing layer). */
typedef struct {
    int32_t ndim;              /* 2 (TMz) or 3 */
    int32_t nx, ny, nz;        /* cells incl. CPML, each >= 3; nz = 1 for ndim 2 */
    double dx, dy, dz, dt;     /* SI units; dz ignored for ndim 2 */
    const float *eps_r;        /* host, nx*ny*nz, >= 1, finite; NULL => 1 */
    const float *mu_r;         /* host, nx*ny*nz, >= 1, finite; NULL => 1 */
    const float *sigma;        /* host, nx*ny*nz, >= 0 S/m, finite; NULL => 0 */
    fdtd_cpml cpml;
    void *stream;              /* hipStream_t to enqueue on; NULL => null stream */
    const fdtd_allocator *allocator; /* NULL => hipMalloc / hipFree */
} fdtd_desc;

typedef struct fdtd_sim fdtd_sim;

/* Build a simulation with the implicit Yee graph: validates the
 * description, folds the edge weights of Prop. 1 (Ca = A-/A+,
 * Cb = dt/(A+ eps), Db = dt/mu, CPML b, c, 1/kappa and 1/d) into per-cell
 * and per-axis float32 tables, allocates zeroed fields.  Input arrays are
 * copied; the caller keeps them.  Errors: FDTD_EINVAL (sizes, steps, maps,
 * CPML thickness 2*npml >= n on an axis), FDTD_EUNSTABLE, FDTD_ENOMEM,
 * FDTD_EDEVICE.  On error *out is NULL. */
int fdtd_create(const fdtd_desc *desc, fdtd_sim **out);

/* Build the same simulation as an explicit graph (ndim 2 only): node order
 * of Prop. 1 (t = 2i+1+nx(3j+1) for Ez, u = i+3j nx for Hx, q = 2i+nx(3j+1)
 * for Hy) with the CPML auxiliary values appended as extra nodes, one CSR
 * matrix per layer (rows = nodes the layer updates, weights = the fixed
 * coefficients of Eq. 7-9 on the previous state).  Every other call works
 * the same on the result. */
int fdtd_create_graph(const fdtd_desc *desc, fdtd_sim **out);

/* Release all device memory (synchronises the stream).  NULL is accepted. */
int fdtd_destroy(fdtd_sim *sim);

/* Point source on an E component (FDTD_EZ for ndim 2) at cell ijk[0..ndim).
 * params as in the FDTD_SRC_* comment (3 doubles, 4 for MODGAUSS;
 * ignored for TABLE).
 * A new call replaces the previous source; kind < 0 removes it.  The cell
 * must not be on a PEC wall plane of that component.  FDTD_EINVAL. */
int fdtd_set_source(fdtd_sim *sim, int component, const int32_t *ijk, int kind,
                    const double *params, const float *table, int64_t n_table);

/* Soft source on every cell of the box [lo, hi) (lo, hi: ndim int32 each,
 * host), all with the same waveform: a line source when one extent exceeds
 * 1 (the paper uses line sources in Sec. V-B without a formula), a plane or
 * volume source otherwise.  Same kinds, parameters and rules as
 * fdtd_set_source (which is this call with hi = lo + 1); the box must lie in
 * the grid, be non-empty and avoid the PEC walls of the component.
 * FDTD_EINVAL. */
int fdtd_set_source_box(fdtd_sim *sim, int component, const int32_t *lo, const int32_t *hi, int kind,
                        const double *params, const float *table, int64_t n_table);

/* Frequency-domain monitor (the paper motivates frequency-domain responses,
 * Sec. I, without a formulation): running discrete Fourier transform of
 * `component` on every cell of the box [lo, hi) (ndim int32 each, host) at
 * the nf frequencies freqs (Hz, >= 0, host): after every step n, from this
 * call on,
 *   X_q[c] += F^{n+1}[c] exp(-2 pi i f_q t_n) dt,
 * t_n = (n+1) dt for an E component and (n+1/2) dt for an H component (the
 * sample's time on the leapfrog grid), summed in FP64.  nf in [0, 16]; a
 * call replaces the monitor (nf = 0 removes it).  While a monitor is set,
 * fdtd_step advances one step per pass (the multi-step kernels do not keep
 * the intermediate steps), and fdtd_step_profile, fdtd_autotune and
 * fdtd_adjoint_eps return FDTD_ESTATE; fdtd_reset zeroes the sums.
 * FDTD_EINVAL for a bad box, component or frequency. */
int fdtd_set_dft(fdtd_sim *sim, int component, const int32_t *lo, const int32_t *hi, int32_t nf,
                 const double *freqs);

/* The monitor's sums: re, im host arrays [nf][box cells] (cells in the
 * box's row-major order, last axis fastest); nsteps (optional) = steps
 * summed.  re = im = NULL: only nsteps.  FDTD_ESTATE without a monitor. */
int fdtd_get_dft(fdtd_sim *sim, double *re, double *im, int64_t *nsteps);

/* Specific absorption rate (W/kg) from the monitor's sums, the monitored E
 * component's share: sar[q][c] = sigma_c |X_qc|^2 / (2 rho_c norm_q^2),
 * X_qc = re + i im of fdtd_get_dft, sigma_c the cell's conductivity (S/m,
 * the material map), rho_c its mass density.  The time-averaged power per
 * unit mass that a time-harmonic field of complex amplitude X deposits
 * (the paper estimates SAR in layered tissue, Sec. V-B); dividing the
 * transient's sums by the source spectrum |S(f_q)| (norm_q) gives it per
 * unit source amplitude.  rho: host float [box cells] (finite, > 0), box
 * order as fdtd_get_dft; norm: host double [nf] (finite, > 0) or NULL
 * (all 1); sar: host float [nf][box cells], written.  Synchronises.
 * FDTD_ESTATE without a monitor; FDTD_EINVAL for a monitor on an H
 * component or a bad rho or norm. */
int fdtd_dft_sar(fdtd_sim *sim, const float *rho, const double *norm, float *sar);

/* Probe cells (ijk: n*ndim int32, host) sampled on `component` after every
 * step: the waveform at chosen points that the paper records from each
 * run (Sec. V-A, the time-domain waveforms of its Fig. 2).  Replaces
 * earlier probes and clears the record.  n <= 4096; cells inside the grid,
 * else FDTD_EINVAL. */
int fdtd_set_probes(fdtd_sim *sim, int component, const int32_t *ijk, int32_t n);

/* Enqueue n >= 0 leapfrog steps on the handle's stream (asynchronous):
 * each step is the two message-passing layers of Prop. 2 (Sec. IV-A), the
 * H layer then the E layer, with the CPML terms, then the soft source and
 * the probe samples.  The kernel configuration (fdtd_set_kernel) decides
 * how steps are grouped into passes over memory; the result is the same
 * leapfrog.  FDTD_EINVAL for n < 0; errors of earlier asynchronous work
 * surface at the next synchronising call. */
int fdtd_step(fdtd_sim *sim, int64_t n);

/* Copy the probe record (the waveforms of Sec. V-A) to host memory
 * out[p*cap + s] for the samples s < min(cap, recorded) of probe p, sample
 * s being the field after step s since the probes were set;
 * *n_recorded = samples recorded since then.  Synchronises.  out may be
 * NULL to query; FDTD_EINVAL for cap < 0. */
int fdtd_probe(fdtd_sim *sim, float *out, int64_t cap, int64_t *n_recorded);

/* fdtd_probe for callers that cannot allocate device memory (code running
 * while other streams capture a HIP graph, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, result and synchronisation as
 * fdtd_probe, but the records are packed in a fixed device array of the
 * library (16 MiB per device, held until the process ends) instead of a
 * block allocated per call, and no device memory is allocated or freed.
 * Limit: probes x min(cap, recorded) <= 4194304 floats, else FDTD_EINVAL
 * (nothing copied; read in several calls or use fdtd_probe).  All calls on
 * one device share that array: calls that overlap on one device (from
 * several threads, or on several streams) race and must be serialised by
 * the caller. */
int fdtd_probe_noalloc(fdtd_sim *sim, float *out, int64_t cap, int64_t *n_recorded);

/* Copy one component (nx*ny*nz float32, same layout as the maps) to dst:
 * the field snapshots of Sec. V-A (Fig. 2).  E components hold step n, H
 * components step n - 1/2 after n steps (the leapfrog staggering of Eq.
 * 7-9).  dst_on_device != 0: dst is device memory (caller-owned), the copy
 * is enqueued on the stream; else host memory and the call synchronises.
 * FDTD_EINVAL for a component the grid does not have (2D: Ez, Hx, Hy). */
int fdtd_get_field(fdtd_sim *sim, int component, void *dst, int dst_on_device);

/* Overwrite one component (tests, resume).  Same layout and flag. */
int fdtd_set_field(fdtd_sim *sim, int component, const void *src, int src_on_device);

/* Whole-state checkpoint and resume (a run continued on another handle of
 * the same problem gives the same bits as an uninterrupted run).  The
 * state is everything a step reads: all field components and every CPML
 * auxiliary array of the current state (the split-field PML: also Ezy;
 * the explicit graph form: its node vector), and the step count, which
 * fixes the source sample of the next step.  Probe records and
 * frequency-domain sums are not part of it.
 *   fdtd_state_bytes: size of the saved state in bytes (a 64-byte header,
 *     then the arrays as float32).
 *   fdtd_save_state: write it to dst (caller-owned, fdtd_state_bytes long;
 *     device memory if dst_on_device, else host).  Synchronises.
 *   fdtd_load_state: replace this handle's state by a saved one; the grid,
 *     absorbing layer, split flag and form must match (FDTD_EINVAL
 *     otherwise, state unchanged).  The probe record restarts empty.
 *     Synchronises. */
int fdtd_state_bytes(fdtd_sim *sim, int64_t *bytes);
int fdtd_save_state(fdtd_sim *sim, void *dst, int dst_on_device);
int fdtd_load_state(fdtd_sim *sim, const void *src, int src_on_device);

/* Zero all fields, auxiliary CPML values, the probe record and the step
 * counter. */
int fdtd_reset(fdtd_sim *sim);

/* Number of steps taken since creation / reset. */
int fdtd_steps_done(const fdtd_sim *sim, int64_t *n);

/* FDTD_ENONFINITE if any field value is NaN or Inf, else FDTD_OK.
 * Synchronises. */
int fdtd_check_finite(fdtd_sim *sim);

/* Replace eps_r (and optionally sigma, may be NULL => unchanged) on the box
 * [lo[d], hi[d]) (host arrays in box order, last axis contiguous) and refold
 * the coefficients there.  Fields are kept. */
int fdtd_set_material(fdtd_sim *sim, const int32_t *lo, const int32_t *hi,
                      const float *eps_r, const float *sigma);

/* Kernel selection for the implicit-graph stepper.
 *  variant: 0 = auto (autotuned or default), 1 = two-pass reference
 *           (separate H and E kernels, in place), 2 = fused single pass
 *           (one kernel per step, double-buffered state), 3 = several
 *           leapfrog steps per pass over memory, 4 = (2D) the whole grid
 *           in one workgroup, its state in registers for all the steps of
 *           an fdtd_step call, the two layers of a step separated by
 *           workgroup barriers: grids without CPML or mu_r map, ny <= 1024
 *           and at most 16 rows per band of ny (rounded up to 64) columns
 *           (16384 cells at most, e.g. 128 x 128), at most 64 probes (an
 *           fdtd_step call with more probes runs variant 2's single
 *           steps); the default where it applies.  3D: every tile
 *           advances two steps in one kernel (state n+1 never leaves the
 *           chip, the x/y-CPML auxiliary values of step n+1 excepted: they
 *           pass through a third state set, allocated on first use, 24 B
 *           per cell plus the CPML auxiliary values); tiles whose
 *           dependency cone stays clear of the x and y CPML slabs run a
 *           kernel without x/y-CPML code.  With tile[1] = 1 the tiles near
 *           the x/y slabs take two fused single steps through the third
 *           set instead.  An odd remainder of fdtd_step's n is one single
 *           step.
 *  tile[0..3]: variant-specific tile sizes (0 = default).
 *  tb: 0 or 1, except for 2D multi-step passes (variant 3 on a 2D grid),
 *    where tb >= 2 TB, a multiple of 2 TB and at most 1024, replays a
 *    captured HIP graph of tb steps (tb / TB passes and a device step
 *    counter, so one graph serves any step range) for the whole multiples
 *    of tb in fdtd_step's n; for grids whose pass costs about as much as its
 *    launch.  The graph is captured on a stream of the library on first use
 *    and again when the tile lists change.
 *    2D fused: tile[0] = V (1, 2 or 4 consecutive y cells per lane; ny % V
 *    must be 0), tile[1] = TX (x rows marched by one wavefront).
 *    3D fused: tile[0] = V (1, 2 or 4 consecutive z cells per thread;
 *    nz % V must be 0); tile[2] = x planes marched by one workgroup (0 =
 *    16, at most 4096); tile[1] and tile[3] must be 0.
 *    3D two-step: as 3D fused with V = 4; also nz <= 512, at most 64
 *    z-CPML cells in all, and no 4-cell z group holding cells of both z
 *    slabs; tile[1] = 0 (tiles near the x/y slabs in the two-step kernel)
 *    or 1 (as two single steps); tile[2] = x planes per interior tile (0:
 *    with tile[1] = 0, the length whose tile list a model of the
 *    device's dispatch finishes first, 16 .. 128; with tile[1] = 1, 16);
 *    tile[3] = x planes per tile of the tiles near the x/y slabs (0 = 16,
 *    at most 4096).
 *    2D multi-step (variant 3 on a 2D grid): tile[0] = V (1, 2 or 4; ny % V
 *    must be 0; 0 = 1), tile[1] = TX (rows per tile, 1..65536; 0 = 4), tile[2] =
 *    TB (leapfrog steps per pass: 2 or 4; 0 = 4), tile[3] = rows per tile
 *    of the tiles near a CPML slab (0 = TX; at most 65536).  Each
 *    wavefront advances its rows and columns TB steps, recomputing the
 *    neighbouring rows and columns it needs; an n not divisible by TB ends
 *    with single steps.  The tiles near a slab run on a second stream of
 *    the library, forked from and joined back to the simulation's stream
 *    within each pass.  The default chunk depends on the grid (16-32 rows
 *    where the interior tiles then fill the device once, else 4 or 8).
 * FDTD_EINVAL for unknown or unsupported combinations. */
typedef struct {
    int32_t variant;
    int32_t tile[4];
    int32_t tb;
} fdtd_kernel_config;

int fdtd_set_kernel(fdtd_sim *sim, const fdtd_kernel_config *cfg);
int fdtd_get_kernel(const fdtd_sim *sim, fdtd_kernel_config *cfg);

/* Time every candidate configuration on this grid for `trial_steps` steps
 * and keep the fastest (the state is saved before and restored after).
 * The choice is cached in the JSON file named by $GEMFDTD_TUNE_CACHE (if
 * set) keyed by device, dimensions and material flags.  out may be NULL. */
int fdtd_autotune(fdtd_sim *sim, int32_t trial_steps, fdtd_kernel_config *out);

/* Device time in milliseconds of the kernels enqueued by the last
 * fdtd_step call, measured with HIP events on the handle's stream
 * (synchronises).  *launches receives the number of kernel launches. */
int fdtd_last_step_time(fdtd_sim *sim, float *ms, int64_t *launches);

/* Per-launch timing of the step.  Advances the state by `steps` steps like
 * fdtd_step, with a HIP event pair around every kernel launch of the 3D
 * fused step (the interior launch and the one of the tiles that touch an x
 * or y CPML slab; with the two-step pass: the first single-step launches,
 * the two-step launch, the second single-step launches, each step pair
 * timed as one unit), or around the whole step for the other steppers, and
 * writes one entry per launch (at most `max`) with the mean duration over
 * the units (steps, or step pairs; an odd last step of a two-step run is
 * not timed); *n receives the number of entries.  cells: cells the entry
 * updates; psi: CPML auxiliary values it updates; cpml: 0 no CPML code, 1
 * z-slab code only, 2 x/y (and z) slab code, -1 a whole step; launches:
 * kernel launches in the entry; steps: leapfrog steps the entry advances
 * its cells by (1, or 2 for the two-step launch).  The events add a small
 * gap between launches. */
typedef struct {
    float ms;
    int64_t cells;
    int64_t psi;
    int32_t cpml;
    int32_t launches;
    int32_t steps;
} fdtd_launch_stat;
int fdtd_step_profile(fdtd_sim *sim, int32_t steps, fdtd_launch_stat *out, int32_t max,
                      int32_t *n);

/* --------------------------------------------------------------------- */
/* Batched form: many independent 2D problems of different sizes advanced  */
/* together, one launch per time block over a packed arena, captured in a  */
/* HIP graph.                                                              */
/* --------------------------------------------------------------------- */
typedef struct fdtd_batch fdtd_batch;

/* descs[0..n) as for fdtd_create (ndim 2; stream and allocator of descs[0]
 * are used for the whole batch).  dt may differ per problem. */
int fdtd_batch_create(const fdtd_desc *descs, int32_t n, fdtd_batch **out);
int fdtd_batch_destroy(fdtd_batch *b);
int fdtd_batch_set_source(fdtd_batch *b, int32_t problem, const int32_t *ijk, int kind,
                          const double *params, const float *table, int64_t n_table);
int fdtd_batch_set_probes(fdtd_batch *b, int32_t problem, const int32_t *ijk, int32_t n);
/* Enqueue n steps of every problem. */
int fdtd_batch_step(fdtd_batch *b, int64_t n);
/* Kernel configuration of the batch: tb leapfrog steps per pass (1, 2 or
 * 4; 1 = single steps only), tx rows per wavefront tile (1..65536), vmax
 * the widest vector of columns per lane (1, 2 or 4; each problem takes the
 * widest its row length allows), txo rows per tile of the tiles near a
 * CPML slab (0 = tx).  Default 4, 16, 1, 0.  Synchronises; the state is
 * kept.  FDTD_EINVAL for other values (the configuration is then
 * unchanged). */
int fdtd_batch_set_kernel(fdtd_batch *b, int32_t tb, int32_t tx, int32_t vmax, int32_t txo);
/* Autotuner of the batch: time every candidate configuration of
 * fdtd_batch_set_kernel (tb in {4, 2}, tx in {8, 16, 32}, vmax in {1, 2,
 * 4}, txo in {0, 4, 8} below tx) for trial_steps steps (8..4096; 64 runs one
 * captured graph) after an 8-step warm-up, and keep the fastest.  The
 * problems' state, step count and probe record lengths are saved before and
 * restored after (the batch continues as if the call had not been made).
 * The choice is cached in the JSON file named by $GEMFDTD_TUNE_CACHE (if
 * set) under the device and the batch's size mix (count, cells, the sorted
 * list of dimensions and material kinds) and reused without timing.
 * out (4 int32, may be NULL): the chosen tb, tx, vmax, txo.  Synchronises.
 * Device memory: a copy of the state while it runs. */
int fdtd_batch_autotune(fdtd_batch *b, int32_t trial_steps, int32_t *out);
int fdtd_batch_probe(fdtd_batch *b, int32_t problem, float *out, int64_t cap,
                     int64_t *n_recorded);
int fdtd_batch_get_field(fdtd_batch *b, int32_t problem, int component, void *dst,
                         int dst_on_device);
int fdtd_batch_last_step_time(fdtd_batch *b, float *ms, int64_t *launches);
/* Total cells of all problems. */
int fdtd_batch_cells(const fdtd_batch *b, int64_t *cells);

/* --------------------------------------------------------------------- */
/* Adjoint: gradient of a probe-energy loss with respect to eps_r.         */
/* --------------------------------------------------------------------- */
/* Starting from the zero state, run T steps with the handle's source,
 * evaluate L = sum_p sum_{m in (n0, n1]} E^m[probe p]^2 (E^m = probe sample
 * m-1 of the handle's probes), and compute dL/d eps_r on the box
 * design = {i0, i1, j0, j1} (ndim 2) by the discrete adjoint: the
 * transposed E and H layers run backward in time.  The forward pass keeps a
 * full-state checkpoint every `ckpt_interval` steps (<= 0 => ceil(sqrt T))
 * and recomputes each segment but the last before its adjoint sweep (the
 * forward pass keeps the last segment's design-cell values).  Device
 * memory: the checkpoints plus 8 B per design cell and step of one
 * segment; ckpt_interval >= T runs no recompute and holds the values of
 * all T steps.
 * loss_out (host, may be NULL); grad_dev: device float32
 * [(i1-i0)*(j1-j0)], written.  On return the handle holds the forward state
 * after T steps and the probe record of the forward run.  FDTD_EINVAL
 * (arguments) leaves the handle unchanged; after FDTD_ENOMEM (checkpoint or
 * design buffers) or FDTD_EDEVICE the handle is usable, every block the
 * call took is released, and its fields may have been reset to zero. */
int fdtd_adjoint_eps(fdtd_sim *sim, int64_t T, int64_t n0, int64_t n1,
                     const int32_t *design, int32_t ckpt_interval, double *loss_out,
                     float *grad_dev);

/* The same adjoint run with the gradients with respect to eps_r and to the
 * conductivity sigma on the design box (the learnable-components direction
 * the paper points to, Sec. I: every per-cell edge weight of the E layer
 * depends on both).  grad_eps_dev, grad_sigma_dev: device float32
 * [(i1-i0)*(j1-j0)], either may be NULL (not both).  fdtd_adjoint_eps is
 * this call with grad_sigma_dev = NULL.  dL/d sigma is per S/m. */
int fdtd_adjoint(fdtd_sim *sim, int64_t T, int64_t n0, int64_t n1, const int32_t *design,
                 int32_t ckpt_interval, double *loss_out, float *grad_eps_dev, float *grad_sigma_dev);

/* Measurement: enqueue a device-to-device copy of `bytes` bytes from src
 * to dst (device pointers, both and bytes multiples of 16, not
 * overlapping) on `stream` (hipStream_t, NULL: null stream) with the
 * library's copy kernel, one 16-byte vector per thread.  Its rate (bytes
 * read plus written per second) is the practical HBM ceiling that the
 * stepping kernels are reported against next to the published peak.
 * Asynchronous; FDTD_EINVAL for misaligned or NULL arguments. */
int fdtd_stream_copy(void *dst, const void *src, size_t bytes, void *stream);

/* The same adjoint run with the gradient with respect to the H layer's
 * per-cell weight as well: dL/d mu_r on the design box (Db = dt/(mu0 mu_r)
 * weighs every message into an H node, Eq. 8-9; the paper's learnable
 * components, Sec. I and VI).  Hx -= Db bx and Hy += Db by at every step, so
 * dL/d mu_r = (Db / mu_r) sum over steps of (aHx bx - aHy by), with aHx,
 * aHy the adjoints of Hx, Hy after the step's H layer; the brackets bx, by
 * are rebuilt from the captured Ez of the design box and one row and
 * column beyond it.  grad_mu_dev: device float32 [(i1-i0)*(j1-j0)] or
 * NULL; any of the three may be NULL, not all.  With grad_mu_dev the
 * design box must lie clear of the CPML slabs (FDTD_EINVAL otherwise).
 * fdtd_adjoint is this call with grad_mu_dev = NULL. */
int fdtd_adjoint_grads(fdtd_sim *sim, int64_t T, int64_t n0, int64_t n1, const int32_t *design,
                       int32_t ckpt_interval, double *loss_out, float *grad_eps_dev, float *grad_sigma_dev,
                       float *grad_mu_dev);

/* Thread-local text of the calling thread's last failure ("" if none). */
const char *fdtd_last_error(void);

/* Library version string. */
const char *fdtd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GEMFDTD_H */
