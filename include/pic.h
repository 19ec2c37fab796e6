/*
 * pic.h - C ABI of the MI355X (gfx950) particle-in-cell hot path.
 *
 * The library advances a relativistic 3D3V particle-in-cell plasma on one GPU:
 * field gather (CIC, TSC or PCS shape on Yee-staggered E, B; standard or
 * Galerkin), relativistic Boris push, Esirkepov charge-conserving current
 * deposition and the Yee FDTD field update, on particles kept sorted into
 * 8x8x4-cell supercells ("frames" of 256 slots per supercell), in FP32 or FP64,
 * plus a Monte Carlo electron-impact ionisation step whose rates come from an
 * exact FP64 Gauss-Laguerre quadrature, a small learned surrogate or a table.  The paper names these methods for its benchmark
 * (section "Evaluation": Boris pusher, Esirkepov current solver, Yee field
 * solver, separable field interpolation, 3D3V, TSC shape) and describes the
 * supercell / frame data structure and the block-per-supercell mapping
 * (section "Preliminaries", PIConGPU); the ionisation step is the Monte Carlo
 * atomic-physics step of its introduction.
 *
 * Units are normalised: c = eps0 = 1, e = m_e = 1, n0 = 1 (omega_p = 1); grid
 * positions are in cell units along each axis; momenta are u = gamma v / c.
 *
 * Conventions shared by every call:
 *   - Every function returns an int status: PIC_OK (0) or a negative
 *     pic_status code.  No C++ exception crosses this boundary.  On error,
 *     pic_last_error() returns a message for the handle (or for the failed
 *     pic_init when passed NULL).
 *   - Argument errors are detected on the host before any GPU work, so they
 *     can be exercised without a GPU.
 *   - A handle is bound to one HIP stream (the hip_stream given to pic_init,
 *     NULL = the default stream).  All GPU work of a call is enqueued on that
 *     stream.  Handles are not thread-safe.
 *   - Device buffers belong to the library: they come from the caller's
 *     allocator (pic_alloc_t) or from hipMalloc, and are released by
 *     pic_destroy.  Host buffers passed to get/set calls belong to the caller.
 *
 * Field arrays on the host are FP32, component-major:
 *   F[c * N + i + nx * (j + ny * k)],  c = 0,1,2 (x,y,z),  N = nx*ny*nz,
 * at the Yee locations Ex (i+1/2,j,k), Ey (i,j+1/2,k), Ez (i,j,k+1/2),
 * Bx (i,j+1/2,k+1/2), By (i+1/2,j,k+1/2), Bz (i+1/2,j+1/2,k); J as E.
 * B excludes the uniform background b0, which is added at gather time.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_ABI_VERSION 7
#define PIC_MAX_SPECIES 4
#define PIC_MAX_ZSTATES 8
#define PIC_LOTZ_SHELLS 3
#define PIC_SUPERCELL_X 8
#define PIC_SUPERCELL_Y 8
#define PIC_SUPERCELL_Z 4

enum pic_status {
    PIC_OK = 0,
    PIC_ERR_ARG = -1,       /* invalid argument (detected before any launch) */
    PIC_ERR_OOM = -2,       /* allocator returned NULL */
    PIC_ERR_HIP = -3,       /* a HIP runtime call failed */
    PIC_ERR_CAPACITY = -4,  /* a supercell's frames or migration buffers overflowed */
    PIC_ERR_CFL = -5,       /* a particle moved one cell or more in one step, or went non-finite */
    PIC_ERR_NONFINITE = -6, /* NaN or Inf found in a field */
    PIC_ERR_STATE = -7      /* call not valid in the handle's current state */
};

/* Particle shape: the B-spline assignment functions of order 1 (CIC), 2 (TSC)
 * and 3 (PCS), used for both the field gather and the Esirkepov deposit. */
typedef enum { PIC_SHAPE_CIC = 1, PIC_SHAPE_TSC = 2, PIC_SHAPE_PCS = 3 } pic_shape_t;
typedef enum { PIC_LAYOUT_UNIFORM = 0, PIC_LAYOUT_SHEAR = 1, PIC_LAYOUT_BEAMS = 2 } pic_layout_t;
/* Ionisation rate: the exact quadrature, the learned surrogate, or a table in
 * ln kT read by cubic interpolation (see pic_ionize). */
typedef enum { PIC_RATE_EXACT = 0, PIC_RATE_MLP = 1, PIC_RATE_TABLE = 2 } pic_rate_mode_t;
/* Real type of particles, fields and currents on the device.  FP64 is the
 * double-precision variant of the PIC cycle that the paper benchmarks beside
 * single precision (section "Evaluation"): the same kernels instantiated in
 * double, with the current tile accumulated by native FP64 LDS atomics and
 * flushed by FP64 global atomics.  Ionisation needs FP32. */
typedef enum { PIC_PRECISION_FP32 = 0, PIC_PRECISION_FP64 = 1 } pic_precision_t;
/* Field gather: STANDARD interpolates every component with the particle's
 * shape on all three axes at its own Yee location; GALERKIN uses the shape
 * one order lower along each axis on which the component is staggered
 * (E_d along d, B_d along the two others; order 0 is the nearest node). */
typedef enum { PIC_GATHER_STANDARD = 0, PIC_GATHER_GALERKIN = 1 } pic_gather_t;

/* Periodic grid.  nx, ny, nz must be positive multiples of 8, 8, 4 (the
 * supercell).  dt must satisfy the 3D Courant limit
 * dt < 1 / sqrt(1/dx^2 + 1/dy^2 + 1/dz^2), which also bounds a particle's
 * displacement to under one cell per step. */
typedef struct {
    int32_t nx, ny, nz;
    int32_t precision;  /* pic_precision_t (0: FP32) */
    double dx, dy, dz, dt;
    double b0[3];       /* uniform background magnetic field */
    double rho_bg;      /* immobile neutralising background charge density (in e n0) */
    uint64_t seed;      /* Philox key for every random draw */
    double n_ref_cm3;   /* physical density of n0 = 1, used only by ionisation */
    int32_t gather;     /* pic_gather_t (0: standard) */
    int32_t options;    /* PIC_OPT_* bits (0: none) */
} pic_grid_t;

/* Options of pic_grid_t.options.
 *
 * PIC_OPT_DETERMINISTIC_J (FP32 only): every supercell's exact 64-bit
 *   fixed-point current tile is added to a 64-bit fixed-point copy of J in
 *   device memory with integer atomics (one scale for all species in a cycle,
 *   2^30 over the largest bound of one particle's contribution), and J is
 *   converted to FP32 once per cycle.  Integer sums do not depend on the order
 *   of the additions, so the cycle's results are bit-reproducible: two runs
 *   from the same state give identical particles and fields.  Without it the
 *   overlapping tiles are added with FP32 atomics, whose order varies.  Costs
 *   24 more bytes per cell and cycle of device traffic (the fixed-point copy
 *   is zeroed and read back) and 24 bytes per cell of memory.
 * PIC_OPT_CONTINUITY: pic_step keeps the FP64 charge density of the state
 *   before its last cycle, so that pic_moments can report that cycle's
 *   continuity residual (pic_moments_t.continuity_max).  Costs one charge
 *   deposit and one extra migration pass per pic_step call. */
#define PIC_OPT_DETERMINISTIC_J 1
#define PIC_OPT_CONTINUITY 2

/* One Lotz subshell of a charge state (Lotz 1968):
 *   sigma_j(E) = a q ln(E/p) / (E p) [1 - b e^{-c (E/p - 1)}]  for E >= p.
 * Subshell 0 is the outermost: its p_ev equals the state's ionization_ev and
 * its q is > 0.  Further subshells have p_ev >= ionization_ev; q = 0 marks an
 * unused slot (all later slots unused too).  a = 4.5e-14 cm^2 eV^2 with
 * b = c = 0 is the plain single-shell form.  Limits: a > 0, 0 <= b <= 1, c >= 0. */
typedef struct {
    double p_ev;           /* binding energy (eV) */
    double a;              /* cm^2 eV^2 */
    double b, c;
    int32_t q;             /* electrons in the subshell */
    int32_t reserved;
} pic_lotz_shell_t;

/* One particle species.
 * Macro-particle weight w = density * dx*dy*dz / ppc.
 * Initial state (t = 0; u is stored at t - dt/2): exactly ppc particles per
 * cell; position = cell corner + 3 Philox uniforms; momentum = drift +
 * u_th * N(0,1) per component from two Box-Muller pairs.  The drift momentum
 * is gamma*beta of drift_beta; layout SHEAR applies +drift for cells with
 * 4j in [ny, 3ny) and -drift elsewhere, BEAMS +drift on even and -drift on odd
 * slots.  coincident_with >= 0 places slot s of every cell on slot s of that
 * (earlier or later) species, whose ppc must be >= this ppc.
 * z_max > 0 gives every particle a charge state Z (starting at z_init); its
 * charge is then charge * Z.  ionization_ev[Z] (Z < z_max) is the ionisation
 * energy of state Z, lotz[Z] its Lotz subshells (below), and ionize_into
 * names the electron species that receives ionisation electrons.
 * max_events (0 or 1: one) caps the ionisations of one ion in one step and
 * energy_loss = 1 makes the electrons of the ion's cell pay the ionisation
 * energy (see pic_ionize). */
typedef struct {
    double charge;         /* in e (per unit Z when z_max > 0) */
    double mass;           /* in m_e */
    double density;        /* in n0 */
    double u_th;           /* thermal momentum spread per component */
    double drift_beta[3];
    int32_t ppc;
    int32_t layout;        /* pic_layout_t */
    int32_t mobile;        /* 0: never pushed (still counted in rho) */
    int32_t coincident_with;
    int32_t z_init, z_max;
    int32_t cap_ppc;       /* frame capacity in particles per cell (0: 3/2 ppc; rounded up to even for TSC and PCS) */
    int32_t ionize_into;   /* species index of ionisation electrons, or -1 */
    double ionization_ev[PIC_MAX_ZSTATES];
    pic_lotz_shell_t lotz[PIC_MAX_ZSTATES][PIC_LOTZ_SHELLS];
    int32_t max_events;    /* ionisations per ion per step (0 or 1: one; at most PIC_MAX_ZSTATES) */
    int32_t energy_loss;   /* 1: the cell's electrons pay the ionisation energy */
} pic_species_t;

/* Device-memory provider.  alloc returns device memory of at least `bytes`
 * bytes aligned to 256 B (NULL on failure; a pointer that is not so aligned
 * is handed back to free and counts as a failure); free releases it. */
typedef struct {
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* ptr, void* user);
    void* user;
} pic_alloc_t;

typedef struct pic_ctx pic_ctx;

/* Create a simulation: allocates frames, fields and scratch, draws the initial
 * particles on the GPU and records the Gauss reference G0 = div E - rho.
 * alloc may be NULL (hipMalloc is used).  hip_stream is a hipStream_t or NULL.
 * Returns PIC_ERR_ARG for invalid sizes, shapes, species or time step, and
 * for an FP64 grid with an ionising species. */
int pic_init(pic_ctx** out, const pic_grid_t* grid, const pic_species_t* species, int n_species,
             pic_shape_t shape, const pic_alloc_t* alloc, void* hip_stream);

/* Advance n >= 0 PIC cycles.  Each cycle: zero J; per mobile species one
 * particle-kernel launch in which each supercell first takes in the particles
 * that arrived from its neighbours in the previous cycle (closing the holes
 * they left), then stages E,B (+guards) in LDS, runs gather + Boris + move +
 * Esirkepov into an LDS current tile flushed once to J, and hands the
 * particles that left it to their destination's arrival list; then B half
 * step, E full step with -J, B half step.  After the last cycle one migration
 * pass takes in the last arrivals, so the frames are dense when the call
 * returns.  Asynchronous on the stream except for one small read of the
 * device error flags at the end (PIC_ERR_CAPACITY, PIC_ERR_CFL). */
int pic_step(pic_ctx* ctx, int n);

typedef struct {
    double w_e;                          /* (1/2) sum |E|^2 dV */
    double w_b;                          /* (1/2) sum |B|^2 dV (b0 excluded) */
    double kinetic[PIC_MAX_SPECIES];     /* sum w m (gamma - 1) at the stored u */
    double kinetic_total;
    double charge_total;                 /* sum rho dV, background included */
    double rho_max;                      /* max |rho| at nodes */
    double gauss_max;                    /* max |(div E - rho) - G0| at nodes */
    double divb_max;                     /* max |div B| at cell centres */
    int64_t count[PIC_MAX_SPECIES];      /* particles per species */
    int64_t step;                        /* cycles taken since init */
    int32_t nonfinite;                   /* number of non-finite E, B entries */
    int32_t reserved;
    /* Continuity residual of the last cycle of the last pic_step call,
     *   max over nodes |div J + (rho^{n+1} - rho^n) / dt|,
     * with div J the backward difference of J (the stencil of div E),
     * rho^n the FP64 charge density at the nodes before that cycle and rho^{n+1}
     * now; zero up to the rounding of J for the Esirkepov deposit.  -1 when the
     * handle lacks PIC_OPT_CONTINUITY, no cycle ran yet, or particles, fields
     * or charge states changed since (pic_set_*, pic_ionize). */
    double continuity_max;
    double j_max;                        /* max |J| over components and cells */
} pic_moments_t;

/* FP64 diagnostics (two-pass reductions on the GPU), synchronous.
 * Returns PIC_ERR_NONFINITE (after filling *out) if a field is not finite. */
int pic_moments(pic_ctx* ctx, pic_moments_t* out);

/* Run state beyond particles and fields, for checkpoint and resume.
 *   step          cycles taken since init; keys the Philox draws of pic_ionize
 *   seed          the Philox key of every draw (pic_grid_t.seed at init)
 *   weight_bound  per species, the bound of |w| that sets the 64-bit
 *                 fixed-point scale of the current tile, 2^30 over
 *                 |q w_bound| max(dx,dy,dz) / (dV dt)
 * A run checkpointed with pic_get_particles / pic_get_fields /
 * pic_get_run_state and resumed on a handle created with the same grid and
 * species, by pic_set_particles, pic_set_fields and then pic_set_run_state,
 * continues exactly as the uninterrupted run (bit for bit with
 * PIC_OPT_DETERMINISTIC_J).  set: PIC_ERR_ARG for step < 0, or for a bound
 * that is not finite or lies below the largest |w| of the species' particles
 * (as known to the handle: from init, pic_set_particles and the electrons
 * pic_ionize adds).  The Gauss reference G0 is not part of it: the resumed
 * handle records its own (pic_mark_reference). */
typedef struct {
    int64_t step;
    uint64_t seed;
    double weight_bound[PIC_MAX_SPECIES];
} pic_run_state_t;

int pic_get_run_state(pic_ctx* ctx, pic_run_state_t* out);
int pic_set_run_state(pic_ctx* ctx, const pic_run_state_t* in);

/* Particle transfer.  Host arrays of `count` entries; positions are global,
 * in cell units, inside [0, n_d).  zstate may be NULL for species without
 * charge states.  get returns particles sorted by id; capacity is the length
 * of the caller's arrays (PIC_ERR_ARG if too small).  set replaces the
 * species' particles (PIC_ERR_CAPACITY if a supercell's frames overflow). */
typedef struct {
    int64_t count;
    int64_t capacity;
    double *x, *y, *z;
    float *ux, *uy, *uz, *w;
    int64_t* id;
    int32_t* zstate;
} pic_particles_view_t;

int pic_particle_count(pic_ctx* ctx, int species, int64_t* count);
int pic_get_particles(pic_ctx* ctx, int species, pic_particles_view_t* v);
int pic_set_particles(pic_ctx* ctx, int species, const pic_particles_view_t* v);

/* Field transfer (host FP32 arrays of 3N, layout above).  NULL skips one. */
int pic_get_fields(pic_ctx* ctx, float* E, float* B, float* J);
int pic_set_fields(pic_ctx* ctx, const float* E, const float* B, const float* J);

/* The same transfers with every real value in FP64 host arrays.  Both
 * families work at either precision; a transfer to an FP32 handle rounds to
 * FP32, one from it widens exactly. */
typedef struct {
    int64_t count;
    int64_t capacity;
    double *x, *y, *z;
    double *ux, *uy, *uz, *w;
    int64_t* id;
    int32_t* zstate;
} pic_particles64_view_t;

int pic_get_particles64(pic_ctx* ctx, int species, pic_particles64_view_t* v);
int pic_set_particles64(pic_ctx* ctx, int species, const pic_particles64_view_t* v);
int pic_get_fields64(pic_ctx* ctx, double* E, double* B, double* J);
int pic_set_fields64(pic_ctx* ctx, const double* E, const double* B, const double* J);

/* Record the current state's div E - rho as the Gauss reference G0.  Called
 * by pic_init; call it again after replacing particles or fields. */
int pic_mark_reference(pic_ctx* ctx);

/* Per-kernel GPU time accounting (HIP events around each launch of pic_step
 * on the handle's stream).  enable = 1 starts accumulating, 0 stops. */
typedef struct {
    double push_ms;        /* particle kernel (gather+push+deposit), all species */
    double migrate_ms;     /* supercell migration */
    double field_ms;       /* J zero + Yee updates */
    int64_t push_launches;
    int64_t push_particles; /* particles processed by the timed push launches */
} pic_timing_t;
int pic_timing(pic_ctx* ctx, int enable, pic_timing_t* out);

/* ------------------------------------------------------------------------
 * Monte Carlo electron-impact ionisation (the Monte Carlo atomic-physics step
 * the paper's introduction adds to the PIC cycle), Lotz model with subshells.
 *
 * For every ion species with z_max > 0 and ionize_into >= 0, per ion with
 * Z < z_max:
 *   - n_e and kT_e of the ion's cell from nearest-grid-point moments of the
 *     electrons of species ionize_into (drift removed):
 *       n_e = (sum w / dV) n_ref_cm3,  kT_e = m_e c^2 (sum w u^2 / sum w - |ubar|^2) / 3;
 *   - rate nu = n_e <sigma v>, <sigma v> the sum over the subshells lotz[Z][j]
 *     of their cross-sections (pic_lotz_shell_t) averaged over a Maxwellian,
 *     evaluated per subshell (p, a, b, c, q) as
 *       vbar (a q / (p kT)) e^{-p/kT} sum_k w_k ln(1 + x_k r) (1 - b e^{-c x_k r}),  r = kT / p
 *     with the 64-point Gauss-Laguerre rule (x_k, w_k) in FP64 (PIC_RATE_EXACT),
 *     by the learned surrogate (PIC_RATE_MLP, see below), or from a table
 *     (PIC_RATE_TABLE): per state Z, h_Z = ln of the subshell sum
 *     sum_j (a_j q_j / p_j) e^{-(p_j - P)/kT} S_j at 1024 points uniform in
 *     ln kT over [1e-2, 1e6] eV, built on the GPU by the same quadrature at
 *     the first call that uses it, read by Catmull-Rom cubic interpolation:
 *     nu = n_e vbar / kT e^{h_Z - P/kT} (interpolation error below 1e-7 in
 *     ln nu); the exact quadrature outside that range;
 *   - p = 1 - exp(-nu dt / omega_p) with omega_p the plasma frequency of
 *     n_ref_cm3; the ion ionises when the Philox uniform of counter
 *     (id, species, 2, step) is below p: Z += 1 and an electron is born at the
 *     ion's position with its momentum and weight, id
 *       N0 + (ion id - first ion id) * z_max + (Z_new - 1)
 *     (N0 = number of particles at t = 0), appended to the same supercell's
 *     frames.  At most one event per ion per call when max_events <= 1.
 *   - max_events = m > 1: successive events in one call.  With n_e and kT_e
 *     frozen, event e (e = 0, 1, ...) adds the waiting time
 *     -ln(1 - u_e) / nu_{Z+e} and happens while the running time stays below
 *     dt / omega_p, for at most m events (and Z < z_max).  u_e is word e % 4
 *     of the Philox block of counter (id, species, 2, step) for e < 4, of
 *     (id, species, 6, step) for e >= 4.  nu_Z of the first event comes from
 *     the chosen mode; later events use the exact quadrature.  Electrons are
 *     born as above, one per event.
 *   - energy_loss = 1: per cell, dE = sum of w * ionization_ev[Z] over its
 *     events; the electrons of species ionize_into that were in the cell
 *     before the call get u <- ubar + f (u - ubar), f = sqrt(max(0,
 *     1 - dE / (3/2 N kT_e))) with N = sum w and ubar, kT_e of the moments
 *     above, so that the cell's kT_e drops by dE / (3/2 N).
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t ions_active;   /* ions with Z < z_max at the start of the call */
    int64_t ionized;       /* ionisation events */
    int64_t fallback;      /* PIC_RATE_MLP / _TABLE: ions rated by the exact quadrature instead */
    int64_t electrons;     /* particles of the receiving species after the call */
    double rate_ms;        /* GPU time of the rate stage (HIP events, handle's stream); -1 when fused */
    double total_ms;       /* GPU time of the whole call */
} pic_ionize_stats_t;

/* One ionisation step for every ionising species.  PIC_ERR_STATE if the
 * handle has no ionising species, or for PIC_RATE_MLP before a surrogate was
 * trained or loaded; PIC_ERR_CAPACITY if a supercell's electron frames are full
 * (an ion keeps only the events whose electrons found a slot).
 * With PIC_RATE_EXACT the moments, the rates and the draw run fused, one
 * workgroup per supercell (rate_ms = -1); PIC_RATE_MLP and PIC_RATE_TABLE
 * run staged as pic_ionize_staged.  Decisions and charge states are those
 * of pic_ionize_staged; the order of the appended electrons within a
 * supercell may differ (it is not defined by either). */
int pic_ionize(pic_ctx* ctx, pic_rate_mode_t mode, pic_ionize_stats_t* out);

/* The same step as three launches over the whole grid: cell moments, the
 * rate of every ion, then the draw and append, with the rate stage timed on
 * its own (rate_ms). */
int pic_ionize_staged(pic_ctx* ctx, pic_rate_mode_t mode, pic_ionize_stats_t* out);

/* Per-cell n_e (cm^-3) and kT_e (eV) of the electrons that species `species`
 * ionises into, as used by pic_ionize (computed now).  Host arrays of
 * nx*ny*nz doubles, cell index i + nx (j + ny k); either may be NULL. */
int pic_cell_moments(pic_ctx* ctx, int species, double* ne_cm3, double* kT_ev);

/* The same moments left on the device: enqueues their computation on the
 * handle's stream and returns the library's own arrays (nx*ny*nz doubles
 * each, same cell index), without a copy or a synchronisation.  They stay
 * owned by the library: the caller must not free or write them, and they
 * are valid until the next pic_ionize, pic_ionize_staged or
 * pic_cell_moments(_device) call on the handle (which overwrite them) or
 * pic_destroy.  Reading them on another stream needs the caller's
 * synchronisation with the handle's stream.  Either pointer may be NULL. */
int pic_cell_moments_device(pic_ctx* ctx, int species, const double** ne_cm3, const double** kT_ev);

/* ln nu (nu in 1/s) for n host samples (kT_e eV, n_e cm^-3, charge state Z of
 * species `species`), by the exact quadrature, the surrogate (with its exact
 * fallback outside the trained range) or the table (built at first use; exact
 * outside its kT range).  Synchronous.  -inf for Z outside [0, z_max) or a
 * non-positive kT_e or n_e. */
int pic_rate_eval(pic_ctx* ctx, pic_rate_mode_t mode, int species, int64_t n, const double* kT_ev,
                  const double* ne_cm3, const int32_t* Z, double* ln_rate);

/* pic_rate_eval for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments and results as pic_rate_eval; the n samples are staged
 * through a static device buffer of the library (one per GPU, about 1.8 MB,
 * held until the process ends, its address taken by pic_init) instead of
 * memory from the handle's allocator, and nothing is allocated.
 * n <= PIC_RATE_EVAL_NOALLOC_MAX, else PIC_ERR_ARG.  Every call on one GPU
 * shares that buffer, so calls that overlap on one GPU (several threads or
 * handles at once) race and must be serialised by the caller.  PIC_RATE_TABLE
 * builds its table at the first use on the handle (a launch into memory taken
 * at pic_init).  Synchronous. */
#define PIC_RATE_EVAL_NOALLOC_MAX 65536
int pic_rate_eval_noalloc(pic_ctx* ctx, pic_rate_mode_t mode, int species, int64_t n, const double* kT_ev,
                          const double* ne_cm3, const int32_t* Z, double* ln_rate);

/* The library's 64-point Gauss-Laguerre rule (weight e^{-x} on [0, inf)),
 * computed on the host at load time by the Golub-Welsch eigenvalue method
 * and refined by Newton steps on the Laguerre recurrence.  Needs no GPU. */
int pic_gauss_laguerre64(double* nodes, double* weights);

/* ------------------------------------------------------------------------
 * Learned ionisation-rate surrogate: 8 -> 64 -> 64 -> 1, SiLU (default) or
 * ReLU activations on both hidden layers.
 *   inputs  (log10 kT_e - 2)/2, (log10 n_e - 21)/2, one-hot of Z (6 states);
 *   output  ln nu = ln nu_prior + mu + s * y, where ln nu_prior is the rate
 *           with e^z E1(z) (z = P/kT) replaced by ln(1 + 1/z):
 *           ln(n_e vbar a q / (P kT)) - z + ln ln(1 + 1/z).
 * Inference runs as a fused BF16-MFMA kernel (BF16 weights and activations,
 * FP32 accumulation and epilogue); inputs outside the trained range
 * [t_min, t_max] x [n_min, n_max] take the exact quadrature.
 * Parameters, flat FP32 (PIC_MLP_NPARAM): W1[64][8], b1[64], W2[64][64],
 * b2[64], W3[1][64], b3[1] (row-major [out][in]).
 * ------------------------------------------------------------------------ */
#define PIC_MLP_NPARAM 4801

/* Hidden-layer activations.  SiLU needs an exp2 and a reciprocal per hidden
 * unit (128 transcendental pairs per ion), ReLU one max. */
#define PIC_MLP_SILU 0   /* z sigmoid(z) */
#define PIC_MLP_RELU 1   /* max(z, 0); derivative 1 for z > 0, else 0 */

typedef struct {
    int64_t n_train;       /* training samples (exact labels generated on the GPU) */
    int32_t batch;         /* minibatch size (multiple of 64) */
    int32_t steps;         /* Adam steps */
    double lr;             /* initial learning rate (cosine decay to lr_final) */
    double lr_final;
    uint64_t seed;         /* Philox key of sample generation, batch draws and init */
    double t_min_ev, t_max_ev, n_min_cm3, n_max_cm3;  /* log-uniform sampling ranges */
    int32_t activation;    /* PIC_MLP_SILU or PIC_MLP_RELU; the trained network keeps it */
    int32_t reserved;      /* 0 */
} pic_mlp_train_cfg_t;

typedef struct {
    double loss_first;     /* minibatch loss of the first step */
    double loss_last;      /* mean minibatch loss of the last 100 steps */
    double mu, s;          /* target standardisation */
    double train_ms;       /* GPU time of data generation + training */
    int64_t steps;
} pic_mlp_report_t;

/* Generate n_train exact-labelled samples on the GPU and train the surrogate of
 * ion species `species` with the library's own forward / backward (BF16 MFMA,
 * FP32 accumulation) and Adam (FP32 master weights) kernels. */
int pic_mlp_train(pic_ctx* ctx, int species, const pic_mlp_train_cfg_t* cfg, pic_mlp_report_t* out);

/* Copy the FP32 master parameters (PIC_MLP_NPARAM floats), (mu, s), the
 * trained range (t/n min/max, 4 doubles) and the activation out / in.  get
 * skips NULL outputs; set needs params and mu_s, keeps the range when range
 * is NULL, and rejects an activation other than PIC_MLP_SILU / PIC_MLP_RELU. */
int pic_mlp_get_params(pic_ctx* ctx, int species, float* params, double* mu_s, double* range, int32_t* activation);
int pic_mlp_set_params(pic_ctx* ctx, int species, const float* params, const double* mu_s, const double* range,
                       int32_t activation);

/* One forward + backward pass of the training kernels (with the species'
 * current activation) on n host samples
 * (features X[n][8], targets t[n]) with the current parameters: writes the
 * mean squared error and its gradient (PIC_MLP_NPARAM floats).  n must be a
 * multiple of 64.  Synchronous. */
int pic_mlp_loss_grad(pic_ctx* ctx, int species, int64_t n, const float* X, const float* t, double* loss,
                      float* grad);

/* Release every device buffer of the handle.  NULL is accepted. */
int pic_destroy(pic_ctx* ctx);

/* Message describing the handle's last error ("" if none); with NULL, the
 * message of the last failed pic_init on this thread. */
const char* pic_last_error(const pic_ctx* ctx);

/* Static facts about the build: ABI version, supercell shape. */
int pic_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PIC_H */
