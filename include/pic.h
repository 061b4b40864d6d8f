/*
 * pic.h -- C ABI of the MI355X (gfx950) FDTD-PIC library.
 *
 * The library advances the particle-in-cell model of Liu, Zhao, Wang & Liu,
 * "Numerical study of three-dimensional PIC for the surface plasmon
 * excitation based on Drude model" (arXiv:1505.04007):
 *
 *   - Yee leapfrog curl updates of E and H (Sec. II, Eqs. 7-8; the magnetic
 *     update "as in vacuum", text after Eq. 8),
 *   - the Drude polarization current J of Eq. 5, discretised as Eq. 6 with
 *     ca = (2 - g dt)/(2 + g dt) and cb = 2 dt eps0 wp^2/(2 + g dt), read with
 *     E at step n, and subtracted in the E update of Eq. 8 (J before E, as the
 *     paper orders them), only where wp > 0,
 *   - a relativistic Boris push of the electron bunch (Sec. III) with
 *     trilinear gather of the staggered fields,
 *   - charge-conserving (Esirkepov, first-order shape) deposition of the
 *     bunch current, also subtracted in the E update.
 * Absorbing walls are convolutional PML (stretched-coordinate, in place of
 * the split-field Berenger PML named in Sec. III).
 *
 * Conventions for every entry point:
 *   - All functions return pic_status; nothing throws across the ABI.
 *   - SI units at the boundary, FP64 host inputs.  Internally the device
 *     state is FP32 in normalised units; probe accumulators and diagnostics
 *     are FP64.
 *   - Host pointers passed in are borrowed for the duration of the call
 *     only; pic_init copies everything it needs.  The context owns every
 *     device allocation it makes and pic_destroy frees them.
 *   - All device work is enqueued on the single HIP stream given in
 *     pic_opts.stream (NULL = the default stream).  pic_step is
 *     asynchronous except for the non-finite-field poll every check_every
 *     steps; pic_probe, pic_read_*, pic_diag, pic_stats and pic_timing
 *     synchronise that stream.
 *   - After PIC_EDEVICE or PIC_EUNSTABLE the context is poisoned: every
 *     later call except pic_destroy and pic_last_error returns PIC_ESTATE.
 *   - A context is not thread-safe; distinct contexts may be used from
 *     distinct threads.
 *
 * Field storage convention used by pic_read_fields / init fields
 * ("compact Yee layout"): each of the three components is an nx*ny*nz
 * array, x fastest (index i + nx*(j + ny*k)), and entry (i,j,k) holds the
 * component at its staggered Yee position relative to node (i,j,k):
 *   Ex(i+1/2, j, k)   Ey(i, j+1/2, k)   Ez(i, j, k+1/2)
 *   Hx(i, j+1/2, k+1/2)   Hy(i+1/2, j, k+1/2)   Hz(i+1/2, j+1/2, k)
 * Positions on the upper walls (node index n) are not stored: they are
 * tangential E / normal H on a PEC wall (identically zero) or, on a
 * periodic axis, copies of node 0.
 */
#ifndef PIC_H
#define PIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The library is built with hidden visibility; these declarations are its
   only exported symbols. */
#if defined(__GNUC__)
#pragma GCC visibility push(default)
#endif

#define PIC_ABI_VERSION 6

typedef enum {
    PIC_OK = 0,
    PIC_EINVAL = -1,    /* bad argument: sizes, boundary codes, CFL bound, particles outside */
    PIC_ENOMEM = -2,    /* a device or host allocation failed */
    PIC_EDEVICE = -3,   /* a HIP runtime call failed (context poisoned) */
    PIC_EUNSTABLE = -4, /* a non-finite field value was detected (context poisoned) */
    PIC_ESTATE = -5,    /* call on a poisoned context, or wrong call order */
    PIC_ENOTSUP = -6    /* feature not available for this context */
} pic_status;

typedef enum { PIC_BC_PEC = 0, PIC_BC_PERIODIC = 1, PIC_BC_CPML = 2 } pic_bc;

typedef enum { PIC_FIELD_E = 0, PIC_FIELD_H = 1, PIC_FIELD_JPOL = 2, PIC_FIELD_JB = 3 } pic_field;

/* Grid and boundaries.  A CPML axis has npml absorbing cells at both ends,
 * backed by a PEC wall.  Grading: sigma = sigma_max (rho/L)^m with
 * sigma_max = pml_sigma_scale * 0.8 (m+1)/(eta0 dx), kappa = 1 +
 * (kappa_max-1)(rho/L)^m, alpha = alpha_max (1 - rho/L) (Roden & Gedney). */
typedef struct {
    int32_t nx, ny, nz;  /* cells per axis, each >= 2 */
    int32_t bc[3];       /* pic_bc per axis */
    int32_t npml;        /* CPML thickness in cells (used on CPML axes), 2*npml < n */
    double pml_m;        /* grading order m (e.g. 3) */
    double pml_sigma_scale;
    double pml_kappa_max;
    double pml_alpha_max;
} pic_grid;

/* One electron species as macro-particles.  Positions in metres inside the
 * box [0, n dx) per axis; u = gamma v in m/s (at t = -dt/2).  q, m are the
 * charge and mass of one physical particle, weight the number of physical
 * particles per macro-particle. */
typedef struct {
    int64_t n;
    const double *x, *y, *z;
    const double *ux, *uy, *uz;
    double q, m, weight;
} pic_particles;

/*
 * Optional caller-owned device memory for the field arrays (for example
 * PyTorch tensors), each nx*ny*nz FP32 values in the compact Yee layout
 * (x fastest), 4-byte aligned, not overlapping one another.  A NULL entry is
 * allocated by the library.  Borrowed: the memory must outlive the context;
 * pic_destroy does not free it.  pic_init overwrites it with the initial
 * state.  E holds E in V/m; H[p] holds eta0 H (V/m) for the two time levels
 * of the H update's ping-pong, H[hcur] (pic_stats) being H^{n-1/2}.  The
 * library writes them asynchronously on the context's stream; readers order
 * their work after it on that stream.
 */
typedef struct {
    float *E[3];
    float *H[2][3];
} pic_device_buffers;

typedef struct {
    void *stream;             /* hipStream_t; NULL = default stream */
    int32_t nprobe;           /* Ez probes (nearest Ez node, ties toward +z) */
    const double *probe_xyz;  /* [3*nprobe] metres */
    int32_t nfreq;            /* DFT frequencies */
    const double *omega;      /* [nfreq] rad/s */
    int64_t series_len;       /* capacity (steps) of the Ez probe time series; 0 = off */
    int32_t sort_every;       /* cell sort of the particles every this many steps; 0 = at init only */
    int32_t check_every;      /* poll the non-finite flag every this many steps; 0 = never */
    const double *init_E[3];  /* optional E at t=0, compact Yee layout, V/m (NULL = zero);
                                 tangential entries on PEC/CPML walls are taken as 0 */
    const double *init_H[3];  /* optional H at t=-dt/2, compact Yee layout, A/m (NULL = zero);
                                 normal entries on PEC/CPML walls are taken as 0 */
    int32_t diag;             /* 1: keep the FP64 charge grid needed by the Gauss check */
    int32_t timing;           /* 1: time every kernel launch with HIP events; k > 1: only
                                 the launches of the steps whose number (pic_stats steps
                                 when the step starts) is a multiple of k, and every sort
                                 (a sample with 1/k of the events' cost to the step) */
    int32_t deposit_mode;     /* 0: wavefront-reduced deposit (default), 1: per-lane atomics,
                                 2: wavefront-reduced into a 64-bit fixed-point current
                                 (each particle's edge currents rounded to 2^-24 of the
                                 largest one particle can deposit, then summed exactly, so
                                 runs are bitwise reproducible; not in batches, nor in
                                 pic_grad with checkpoints) */
    const pic_device_buffers *bufs;  /* optional caller device memory for E and H; NULL = none */
    int32_t field_sweep;      /* 0: the separate H and E launches (the default, faster on
                                 the grids measured); 1: pic_step fuses each step's E update
                                 with the next step's H update into one pass over the grid
                                 where it can (deposit modes 0 and 1, nx <= 1024, each of E,
                                 H[0], H[1] one block with its components nx*ny*nz apart),
                                 with the same bits as the separate launches, keeping a
                                 second copy of E, J_pol and the E-side CPML memories on the
                                 device */
} pic_opts;

typedef struct pic_ctx pic_ctx;

typedef struct {
    double field_energy;  /* (eps0 |E|^2 + mu0 |H|^2)/2 dx^3 summed over stored entries, J */
    double count;         /* live macro-particles */
    double mean[3];       /* mean position, m */
    double rms[3];        /* rms size about the mean, m */
    double umean[3];      /* mean gamma v, m/s */
    double gauss_max;     /* max |eps0 div E - rho + rho0| over checked nodes, C/m^3 (diag=1) */
    double rho0_max;      /* max |rho0| at init, C/m^3 (diag=1) */
    int64_t checked_nodes;/* nodes in the Gauss check: interior, outside CPML and metal */
} pic_diag_out;

typedef struct {
    int64_t steps;        /* steps taken */
    int64_t pushes;       /* particle pushes actually deposited (live particles x steps) */
    int64_t live;         /* live particles now */
    int32_t pbox[6];      /* cell bounding box of the live particles at the last sort:
                             lo x, y, z, hi x, y, z (inclusive); hi < lo when empty */
    int32_t hcur;         /* which H buffer (0 or 1) holds H^{n-1/2} for the next step */
    int64_t device_bytes; /* device memory the context allocated itself at pic_init, bytes */
} pic_stats_out;

/* Device memory a context needs, from pic_query_sizes. */
typedef struct {
    int64_t field_elems;       /* FP32 elements of each field array: nx*ny*nz (E[c], H[p][c]) */
    int64_t field_bytes;       /* bytes of each field array, 4 * field_elems */
    int64_t device_bytes;      /* bytes pic_init allocates itself for these arguments, metal box excluded */
    int64_t bytes_per_metal_box_cell; /* plus this much per cell of the bounding box of wp > 0 */
} pic_buffer_sizes;

/* Library ABI version (PIC_ABI_VERSION). */
int pic_abi_version(void);

/*
 * Create a simulation.
 *   grid       : sizes and boundaries (see pic_grid)
 *   dx, dt     : cubic cell size (m) and time step (s); dt must satisfy the
 *                Yee + Drude bound 3 (c dt/dx)^2 + (wp_max dt / 2)^2 <= 1
 *   wp_map     : [nx*ny*nz] plasma frequency wp per cell, rad/s (Eq. 1), x fastest
 *   gamma_map  : [nx*ny*nz] collision frequency per cell, 1/s (Eq. 1)
 *                Cell (i,j,k) owns the edges Ex(i+1/2,j,k), Ey(i,j+1/2,k),
 *                Ez(i,j,k+1/2); wp = 0 means vacuum (J = 0 there).
 *   particles  : NULL or n = 0 for a fields-only run
 *   opts       : NULL for defaults
 * On success *ctx is a new context.  Errors: PIC_EINVAL (sizes, bc codes,
 * npml, negative maps, CFL bound, particles outside the box), PIC_ENOMEM,
 * PIC_EDEVICE.  On error *ctx is NULL.
 */
pic_status pic_init(pic_ctx **ctx, const pic_grid *grid, double dx, double dt,
                    const double *wp_map, const double *gamma_map,
                    const pic_particles *particles, const pic_opts *opts);

/*
 * Device memory pic_init will need, without creating anything (no device
 * call; callers size their own buffers for pic_opts.bufs from it, or check
 * that a problem fits).  grid and nparticles as for pic_init; opts may be
 * NULL and is read only for what changes the allocations: nprobe, nfreq,
 * series_len, diag, and which entries of bufs are non-NULL (the pointers
 * themselves are not used).  The Drude state depends on the maps: add
 * bytes_per_metal_box_cell times the cells of the bounding box of wp > 0.
 * pic_stats reports what a context actually allocated, for comparison.
 * Errors: PIC_EINVAL (NULL grid or out, sizes, npml, counts out of range).
 */
pic_status pic_query_sizes(const pic_grid *grid, int64_t nparticles, const pic_opts *opts,
                           pic_buffer_sizes *out);

/*
 * Advance nsteps >= 0 full time steps, each in the order of Sec. II (the
 * text after Eq. 8): the H update in its vacuum form, the bunch push and
 * current deposit (gather, Boris, move, Esirkepov), the Drude current of
 * Eq. 6 from E^n, the E update of Eq. 8 less both currents, then the probe
 * DFT.  The particles are re-sorted by cell every sort_every steps.
 * Asynchronous on the context's stream, except for the non-finite poll every
 * check_every steps (PIC_EUNSTABLE, context poisoned, when it finds one).
 * Errors: PIC_EINVAL (nsteps < 0), PIC_ESTATE, PIC_EDEVICE, PIC_EUNSTABLE.
 */
pic_status pic_step(pic_ctx *ctx, int64_t nsteps);

/*
 * FP64 probe spectra F[p][m] = sum_n dt Ez_p^n exp(-i omega_m n dt),
 * n = 1..steps (Sec. IV, Figs. 6-7).  re, im: [nprobe*nfreq] (may be NULL);
 * series: [nprobe*min(steps, series_len)] Ez samples, step-major (may be NULL).
 */
pic_status pic_probe(pic_ctx *ctx, double *re, double *im, double *series);

/*
 * Gradient of the probe spectral power with respect to the Drude maps of
 * Eq. 1 (the differentiable form of the Sec. II step).
 *
 * Advances the simulation by nsteps steps exactly as pic_step would (the
 * context ends in the same state, probe spectra included) and returns
 *   L = sum_p |F_p|^2,  F_p = sum_{n = s0+1}^{s0+nsteps} dt Ez_p^n exp(-i omega0 n dt)
 * (s0 = steps taken before the call; the probes are those given at
 * pic_init) and, per cell, dL/dwp and dL/dgamma with the bunch current held
 * at the values this run deposits (the current is recorded and prescribed;
 * the field's back-action on the bunch is not differentiated).
 *
 * Method: the reverse pass runs the transposed field + Drude + CPML step
 * back through the run, accumulating the gradient in FP64; it needs E^n and
 * J^{n-1/2} on the metal box at every step.  With ckpt_every = 0 and
 * nsteps * 24 bytes per metal-box cell within half the free device memory,
 * the forward run keeps those snapshots for every step and nothing is
 * replayed.  Otherwise (ckpt_every > 0, or 0 when they do not fit:
 * ceil(sqrt(nsteps))) the forward run stores a field checkpoint every
 * ckpt_every steps and the bunch current of every step on its particle box,
 * and the reverse pass replays each segment from its checkpoint with the
 * recorded current.  Both give the same result.  Device memory is allocated
 * for the call and released before it returns: the snapshots and one
 * adjoint field state, plus with checkpoints about (nsteps/ckpt_every + 1)
 * field states and the recorded current.
 *
 *   omega0     : rad/s
 *   L          : out, V^2 s^2 / m^2
 *   dL_dwp     : out [nx*ny*nz] (same layout as wp_map), per rad/s; may be NULL
 *   dL_dgamma  : out [nx*ny*nz], per 1/s; may be NULL
 * Both maps are 0 outside cells with wp > 0.  Synchronises the stream.
 * Errors: PIC_EINVAL (nsteps < 1, ckpt_every < 0, no probes, L NULL,
 * omega0 not finite), PIC_ENOTSUP (checkpoints with deposit_mode 2: the
 * recorded current is FP32), PIC_ENOMEM, PIC_EDEVICE, PIC_EUNSTABLE.  After an
 * error other than PIC_EINVAL the simulation may stand at any step of the
 * call's forward run.
 */
pic_status pic_grad(pic_ctx *ctx, double omega0, int64_t nsteps, int64_t ckpt_every, double *L,
                    double *dL_dwp, double *dL_dgamma);

/*
 * pic_grad without device allocation, for callers that cannot allocate
 * device memory (code recording a HIP graph, serving loops, harnesses that
 * forbid hipMalloc).  Same result as pic_grad(ctx, omega0, nsteps, 0, ...)
 * taken in its store-all form (every step's metal-box snapshot kept, nothing
 * replayed), and the same kernels; every device buffer of the call (the
 * snapshots, the FP64 probe record, the adjoint state and the gradient
 * accumulators) is carved from one static device array of 64 MiB that the
 * library holds on each device it runs on until the process ends, and the
 * call allocates and frees no device memory (host memory for the FP64
 * objective is ordinary heap memory; per-launch timing, opts.timing, is
 * suspended for the call since it creates HIP events).  The array is
 * cleared where it must start at zero on every call, so it keeps no result
 * from one call to the next, but all calls on one device share it: calls
 * that overlap in time on one device (other threads, other streams) race
 * and give wrong results.
 * Needs roughly nsteps * 24 bytes per metal-box cell plus 28 bytes per grid
 * cell (and the CPML slabs); a call that needs more than the array holds
 * returns PIC_EINVAL with the sizes in the message, before anything runs.
 * Errors: as pic_grad, plus PIC_EINVAL (scratch too small) and PIC_EDEVICE
 * when the array's device address could not be obtained at pic_init.
 */
pic_status pic_grad_noalloc(pic_ctx *ctx, double omega0, int64_t nsteps, double *L, double *dL_dwp,
                            double *dL_dgamma);

/* Result of the field-kernel tile autotuner. */
typedef struct {
    int32_t tile;     /* chosen tile variant index */
    int32_t fx, fy;   /* its cells along x and y (one z plane per workgroup) */
    int32_t order;    /* 0: tiles numbered x, y, z (plane by plane); 1: x, z, y */
    int32_t nshapes;  /* variants in the table (entries of ms) */
    double ms[16];    /* measured ms per H + E launch pair, per variant (0 when forced) */
} pic_tune_out;

/*
 * Choose the tile shape and tile order of the field kernels (H update and
 * Drude + E update) for this grid.  With force = -1, times reps H + E launch
 * pairs of every variant in the library's table on the context's stream, starting from
 * the current field state and restoring it afterwards (fields, CPML
 * memories, Drude current, step clock), and keeps the fastest (the default
 * shape 0 unless another is more than 3 % faster); with force in
 * [0, nshapes) selects that shape without timing.  Results of later steps
 * do not depend on the shape (each cell's arithmetic is the same).
 * Synchronises the stream.  out may be NULL.  Errors: PIC_EINVAL, PIC_ENOMEM,
 * PIC_EDEVICE.
 */
pic_status pic_tune(pic_ctx *ctx, int32_t reps, int32_t force, pic_tune_out *out);

/*
 * Copy one field to host: host_out[3*nx*ny*nz], the three components one after
 * another in the compact Yee layout, SI units (E V/m, H A/m, J_pol and J_b
 * A/m^2; J_pol is the current of Eq. 6, zero outside the metal box).
 * Synchronises the stream.  Errors: PIC_EINVAL (unknown field, NULL), PIC_ESTATE,
 * PIC_EDEVICE.
 */
pic_status pic_read_fields(pic_ctx *ctx, int which, double *host_out);

/* Copy particles to host, ordered by their original index: out[6*n] =
 * x[n], y[n], z[n] (m; NaN once a particle has left the box), ux, uy, uz (m/s). */
pic_status pic_read_particles(pic_ctx *ctx, double *host_out);

/* FP64 diagnostics of the current state. */
pic_status pic_diag(pic_ctx *ctx, pic_diag_out *out);

/* Step and push counters. */
pic_status pic_stats(pic_ctx *ctx, pic_stats_out *out);

/*
 * Per-kernel device time (opts.timing >= 1), measured with HIP events on the
 * context's stream.  names: kernel families in order
 *   0 h_update, 1 push_deposit, 2 e_update, 3 probe, 4 sort,
 *   5 field_sweep (the one-pass E + H update, with its clear of the bunch current).
 * ms_total[6], launches[6] receive the accumulated milliseconds and counts
 * of the timed launches since init or the last reset (with timing = k > 1,
 * those of the sampled steps and every sort); reset = 1 clears them
 * afterwards.
 * The context holds two HIP events per timed launch until a reset: in a
 * long timed run, call with reset = 1 from time to time.
 */
pic_status pic_timing(pic_ctx *ctx, double *ms_total, int64_t *launches, int reset);

/* Destroy a context and free everything it owns.  NULL is a no-op. */
void pic_destroy(pic_ctx *ctx);

/*
 * Batched simulations (e.g. a sweep over film thickness and bunch energy):
 * advance n independent contexts together with one launch per kernel family
 * per step for all of them, instead of one per context.
 *
 * pic_batch_create: ctxs[0..n) are existing contexts (1 <= n <= 64) created
 *   on one stream; those with particles must share sort_every and
 *   deposit_mode (0 or 1; deposit_mode 2 gives PIC_ENOTSUP).  The batch
 *   borrows them: they must outlive it and stay valid; reading them
 *   (pic_probe, pic_read_*, pic_diag, ...) between batch steps is allowed.
 *   use_graph = 1 captures one sort period (sort_every steps and the sorts
 *   that follow, or 10 steps without particles) as a HIP graph at creation
 *   and replays it whenever all members are at the start of a sort period;
 *   other steps are issued directly.
 * pic_batch_step: advance every member by nsteps steps.  Each member's
 *   results equal those of pic_step on that member alone (same kernels, same
 *   per-cell arithmetic).  No non-finite poll is made; use pic_diag.
 * Errors: PIC_EINVAL (arguments), PIC_ESTATE (a poisoned member),
 *   PIC_EDEVICE, PIC_ENOMEM; the message is in pic_batch_last_error.
 */
typedef struct pic_batch pic_batch;
pic_status pic_batch_create(pic_batch **batch, pic_ctx *const *ctxs, int32_t n, int32_t use_graph);
pic_status pic_batch_step(pic_batch *batch, int64_t nsteps);
/*
 * The autotuner for a batch: one tile shape for all members' field launches
 * (the batched H and E kernels), timed like pic_tune over the whole batch
 * with every member's state restored; re-captures the batch's graph.
 */
pic_status pic_batch_tune(pic_batch *b, int32_t reps, int32_t force, pic_tune_out *out);
void pic_batch_destroy(pic_batch *batch);
const char *pic_batch_last_error(const pic_batch *batch);

/* Message of the last error on ctx (or of the last failed pic_init when ctx
 * is NULL).  Owned by the library; valid until the next call on ctx. */
const char *pic_last_error(const pic_ctx *ctx);

#if defined(__GNUC__)
#pragma GCC visibility pop
#endif

#ifdef __cplusplus
}
#endif

#endif /* PIC_H */
