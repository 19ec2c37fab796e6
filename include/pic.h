/*
 * pic.h - C ABI of the MI355X (gfx950) particle-in-cell hot path.
 *
 * The library advances a relativistic 3D3V particle-in-cell plasma on one GPU:
 * field gather (CIC or TSC shape on Yee-staggered E, B), relativistic Boris
 * push, Esirkepov charge-conserving current deposition and the Yee FDTD field
 * update, on particles kept sorted into 8x8x4-cell supercells ("frames" of 256
 * slots per supercell), plus a Monte Carlo electron-impact ionisation step
 * whose rates come from an exact FP64 Gauss-Laguerre quadrature or from a
 * small learned surrogate.  The paper names these methods for its benchmark
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

#define PIC_ABI_VERSION 1
#define PIC_MAX_SPECIES 4
#define PIC_MAX_ZSTATES 8
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

typedef enum { PIC_SHAPE_CIC = 1, PIC_SHAPE_TSC = 2 } pic_shape_t;
typedef enum { PIC_LAYOUT_UNIFORM = 0, PIC_LAYOUT_SHEAR = 1, PIC_LAYOUT_BEAMS = 2 } pic_layout_t;
typedef enum { PIC_RATE_EXACT = 0, PIC_RATE_MLP = 1 } pic_rate_mode_t;

/* Periodic grid.  nx, ny, nz must be positive multiples of 8, 8, 4 (the
 * supercell).  dt must satisfy the 3D Courant limit
 * dt < 1 / sqrt(1/dx^2 + 1/dy^2 + 1/dz^2), which also bounds a particle's
 * displacement to under one cell per step. */
typedef struct {
    int32_t nx, ny, nz;
    int32_t reserved0;
    double dx, dy, dz, dt;
    double b0[3];       /* uniform background magnetic field */
    double rho_bg;      /* immobile neutralising background charge density (in e n0) */
    uint64_t seed;      /* Philox key for every random draw */
    double n_ref_cm3;   /* physical density of n0 = 1, used only by ionisation */
} pic_grid_t;

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
 * charge is then charge * Z.  ionization_ev[Z] and lotz_q[Z] (Z < z_max) are
 * the ionisation energy and outer-shell electron count of state Z, and
 * ionize_into names the electron species that receives ionisation electrons. */
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
    int32_t cap_ppc;       /* frame capacity in particles per cell (0: 3/2 ppc) */
    int32_t ionize_into;   /* species index of ionisation electrons, or -1 */
    double ionization_ev[PIC_MAX_ZSTATES];
    int32_t lotz_q[PIC_MAX_ZSTATES];
} pic_species_t;

/* Device-memory provider.  alloc returns device memory of at least `bytes`
 * bytes aligned to 256 B (NULL on failure); free releases it. */
typedef struct {
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* ptr, void* user);
    void* user;
} pic_alloc_t;

typedef struct pic_ctx pic_ctx;

/* Create a simulation: allocates frames, fields and scratch, draws the initial
 * particles on the GPU and records the Gauss reference G0 = div E - rho.
 * alloc may be NULL (hipMalloc is used).  hip_stream is a hipStream_t or NULL.
 * Returns PIC_ERR_ARG for invalid sizes, shapes, species or time step. */
int pic_init(pic_ctx** out, const pic_grid_t* grid, const pic_species_t* species, int n_species,
             pic_shape_t shape, const pic_alloc_t* alloc, void* hip_stream);

/* Advance n >= 0 PIC cycles.  Each cycle: zero J; per mobile species and
 * supercell, stage E,B (+guards) in LDS, gather + Boris + move + Esirkepov
 * into an LDS current tile flushed once to J; migrate particles that left
 * their supercell; B half step, E full step with -J, B half step.
 * Asynchronous on the stream except for one small read of the device error
 * flags at the end (PIC_ERR_CAPACITY, PIC_ERR_CFL). */
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
} pic_moments_t;

/* FP64 diagnostics (two-pass reductions on the GPU), synchronous.
 * Returns PIC_ERR_NONFINITE (after filling *out) if a field is not finite. */
int pic_moments(pic_ctx* ctx, pic_moments_t* out);

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
