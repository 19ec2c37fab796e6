// Internal declarations of the Monte Carlo ionisation step and its rate
// paths (exact quadrature, learned surrogate, table): the per-species Lotz
// tables, the draw arguments and buffers, the launchers each kernel file
// provides, and the device-side Lotz rate shared by the kernels.
#pragma once

#include "pic_device.hpp"

namespace pic {

// ---------------------------------------------------------------- ionisation
constexpr int GL_NODES = 64;                 // Gauss-Laguerre points
constexpr double ME_C2_EV = 510998.95;       // electron rest energy (eV)
constexpr double C_CM_S = 2.99792458e10;     // speed of light (cm/s)
constexpr double LOTZ_A = 4.5e-14;           // Lotz constant (cm^2 eV^2)

// Lotz subshells per charge state Z (subshell 0 the outermost, sp[Z][0] = P[Z]).
struct IonTables {
    double P[PIC_MAX_ZSTATES];                    // ionisation energy of state Z (eV)
    double sp[PIC_MAX_ZSTATES][PIC_LOTZ_SHELLS];  // subshell binding energies (eV)
    double aq[PIC_MAX_ZSTATES][PIC_LOTZ_SHELLS];  // a q (cm^2 eV^2)
    double sb[PIC_MAX_ZSTATES][PIC_LOTZ_SHELLS];  // b
    double sc[PIC_MAX_ZSTATES][PIC_LOTZ_SHELLS];  // c
    int ns[PIC_MAX_ZSTATES];                      // subshells in use
    int z_max;
};

// Ionisation counters (unsigned long long): [CNT_FALLBACK] is the length of
// the fallback list; the active-ion and event counts are striped over
// CNT_STRIPES words each (supercell sc adds to word sc % CNT_STRIPES) so that
// thousands of workgroups do not serialise on one address; the host sums them.
constexpr int CNT_FALLBACK = 2, CNT_STRIPES = 64;
constexpr int CNT_ACTIVE = 8, CNT_FIRED = CNT_ACTIVE + CNT_STRIPES, CNT_WORDS = CNT_FIRED + CNT_STRIPES;

struct DrawArgs {
    uint64_t seed;
    int64_t step;
    int species_index;
    int64_t ion_id_offset;
    int64_t id_base_new;
    double dt_phys;             // dt / omega_p in seconds
    int max_events;             // <= 1: one event per ion; else the waiting-time chain
    int energy_loss;            // 1: accumulate w * P per cell into de
};
// Per-step ionisation buffers the draw and energy-loss kernels share.
struct DrawBuffers {
    const double* ne;           // per cell n_e (cm^-3)
    const double* kT;           // per cell kT_e (eV)
    const double* gl;           // Gauss-Laguerre rule (later events' exact rates)
    const double* mom4;         // per cell N = sum w and mean u (energy loss), or nullptr
    double* de;                 // per cell sum of w * P over the events (energy loss), or nullptr
    int32_t* old_count;         // per supercell electron count before the appends (energy loss), or nullptr
};

// Tabulated rate (PIC_RATE_TABLE): RATE_TABLE_N nodes per charge state,
// uniform in ln kT, covering [RATE_TABLE_TMIN, RATE_TABLE_TMAX] eV.
constexpr int RATE_TABLE_N = 1024;
constexpr double RATE_TABLE_TMIN = 1e-2, RATE_TABLE_TMAX = 1e6;
hipError_t launch_rate_table_build(const IonTables& tab, const double* gl, double* table, hipStream_t st);
// fb_list: one entry per ion slot, for the ions outside the table's range
hipError_t launch_rate_table(const GridView& g, const SpeciesView& ion, const IonTables& tab, const double* ne,
                             const double* kT, double* nu, const double* table, const double* gl,
                             unsigned long long* counters, unsigned long long* fb_list, hipStream_t st);
hipError_t launch_ln_rate_table(int64_t n, const double* kT, const double* ne, const int32_t* Z, const IonTables& tab,
                                const double* table, const double* gl, double* out, hipStream_t st);

// host: the 64-point Gauss-Laguerre rule (nodes; weights through *w)
const double* gauss_laguerre_nodes(const double** w);

// mom4: per cell (sum w, mean ux, uy, uz), or nullptr
hipError_t launch_moments(const GridView& g, const SpeciesView& e, double n_ref_over_dv, double* ne, double* kT,
                          double* mom4, hipStream_t st);
hipError_t launch_rate_exact(const GridView& g, const SpeciesView& ion, const IonTables& tab, const double* ne,
                             const double* kT, double* nu, const double* gl, hipStream_t st);
hipError_t launch_ln_rate_exact(int64_t n, const double* kT, const double* ne, const int32_t* Z, const IonTables& tab,
                                const double* gl, double* out, hipStream_t st);
hipError_t launch_draw_append(const GridView& g, const SpeciesView& ion, const SpeciesView& el, const IonTables& tab,
                              const DrawArgs& a, const double* nu, const DrawBuffers& b, unsigned long long* counters,
                              hipStream_t st);
hipError_t launch_energy_loss(const GridView& g, const SpeciesView& el, const DrawBuffers& b, hipStream_t st);
// The step with the exact rate fused (moments, rate, draw and append per
// supercell in one kernel); ne, kT (and mom4) receive the cell moments as
// the staged step's do.
hipError_t launch_ionize_exact(const GridView& g, const SpeciesView& ion, const SpeciesView& el, const IonTables& tab,
                               const DrawArgs& a, const DrawBuffers& db, double n_ref_over_dv, double* ne, double* kT,
                               double* mom4, unsigned long long* counters, hipStream_t st);

// ---------------------------------------------------------------- surrogate
struct MlpLaunch {
    const float* params;   // FP32 master parameters (PIC_MLP_NPARAM)
    double mu, s;          // target standardisation
    double t_min, t_max, n_min, n_max;
    int act;               // PIC_MLP_SILU or PIC_MLP_RELU
};
struct MlpGen {
    double lt_min, lt_max, ln_min, ln_max;  // log10 ranges of kT (eV) and n_e (cm^-3)
};
struct MlpStep {
    const float* X;        // [n_data][8] features
    const float* t;        // [n_data] standardised targets
    int64_t n_data;
    int batch;             // multiple of 64
    uint64_t draw_seed;    // 0: samples 0..batch-1 in order; else Philox draws
    int64_t step;
    int act;               // PIC_MLP_SILU or PIC_MLP_RELU
};
// fb_list: one entry per ion slot (nsc * cap), for the out-of-range ions
hipError_t launch_rate_mlp(const GridView& g, const SpeciesView& ion, const IonTables& tab, const MlpLaunch& ml,
                           const double* ne, const double* kT, double* nu, const double* gl,
                           unsigned long long* counters, unsigned long long* fb_list, hipStream_t st);
// The exact FP64 rate for the counters[2] ions listed in fb_list.
hipError_t launch_rate_fallback(const GridView& g, const SpeciesView& ion, const IonTables& tab, const double* ne,
                                const double* kT, double* nu, const double* gl, const unsigned long long* fb_list,
                                const unsigned long long* counters, hipStream_t st);
hipError_t launch_ln_rate_mlp(int64_t n, const double* kT, const double* ne, const int32_t* Z, const IonTables& tab,
                              const MlpLaunch& ml, const double* gl, double* out, hipStream_t st);
hipError_t launch_mlp_gen(int64_t n, uint64_t seed, const MlpGen& a, const IonTables& tab, const double* gl, float* X,
                          double* r, hipStream_t st);
hipError_t launch_mlp_standardize(int64_t n, const double* r, double* partial, double* mu_s, float* t, hipStream_t st);
hipError_t launch_mlp_init(uint64_t seed, float* P, float* m, float* v, hipStream_t st);
// A training step's gradient is summed without atomics: each workgroup of
// the step kernel writes its sum (its waves in order) to its own row of a
// partial buffer, MLP_PART_ROWS rows of MLP_PART_STRIDE floats (and its
// squared-error sum to lpart), and the Adam kernel, or launch_mlp_grad, adds
// the rows in row order.  *rows receives the number of rows written.
constexpr int MLP_PART_ROWS = 64;
constexpr int MLP_PART_STRIDE = (PIC_MLP_NPARAM + 63) / 64 * 64;
hipError_t launch_mlp_step(const float* P, const MlpStep& s, float* part, double* lpart, int* rows, hipStream_t st);
// Adam on the master parameters with the summed gradient; *loss = the summed squared error
hipError_t launch_mlp_adam(float* P, const float* part, int rows, const double* lpart, double* loss, float* m, float* v,
                           float lr, float bc1, float bc2, hipStream_t st);
// the summed gradient (PIC_MLP_NPARAM floats) and squared error
hipError_t launch_mlp_grad(const float* part, int rows, const double* lpart, float* grad, double* loss, hipStream_t st);

// Static staging of pic_rate_eval_noalloc (noalloc.hip): one device array per
// GPU, its address taken once per device by noalloc_scratch_setup (with that
// device current) and returned by noalloc_scratch (nullptr before).
struct NoallocStaging {
    double *kT, *ne, *out;
    int32_t* Z;
};
hipError_t noalloc_scratch_setup(int device);
unsigned char* noalloc_scratch(int device);
NoallocStaging noalloc_staging(unsigned char* base);

// ---------------------------------------------------------------- Lotz rate
// One subshell (p, a, b, c, q) with E = p + kT x:
//   <sigma v>_j = vbar (a q / (p kT)) e^{-p/kT} sum_k w_k ln(1 + x_k r) (1 - b e^{-c x_k r}),  r = kT / p,
// FP64; the exponential only where b != 0.
__device__ inline double lotz_sum(double r, double b, double c, const double* glx, const double* glw)
{
    double s = 0.0;
    if (b == 0.0) {
#pragma unroll 8
        for (int k = 0; k < GL_NODES; ++k) s = fma(glw[k], log1p(glx[k] * r), s);
    } else {
#pragma unroll 4
        for (int k = 0; k < GL_NODES; ++k) {
            const double xr = glx[k] * r;
            s = fma(glw[k] * log1p(xr), 1.0 - b * exp(-c * xr), s);
        }
    }
    return s;
}

// sum_j (a_j q_j / p_j) e^{-(p_j - P)/kT} S_j over the subshells of state Z, P = P[Z]:
// the state's <sigma v> is vbar / kT e^{-P/kT} times this.
__device__ inline double lotz_shells(double kT, const IonTables& t, int Z, const double* glx, const double* glw)
{
    double acc = 0.0;
    for (int j = 0; j < t.ns[Z]; ++j) {
        const double p = t.sp[Z][j];
        double v = t.aq[Z][j] / p * lotz_sum(kT / p, t.sb[Z][j], t.sc[Z][j], glx, glw);
        if (j > 0) v *= exp(-(p - t.P[Z]) / kT);
        acc += v;
    }
    return acc;
}

__device__ inline double vbar_cm_s(double kT) { return C_CM_S * sqrt(8.0 * kT / (M_PI * ME_C2_EV)); }

__device__ inline double rate_exact(double kT, double ne, const IonTables& t, int Z, const double* glx,
                                    const double* glw)
{
    if (!(kT > 0.0) || !(ne > 0.0)) return 0.0;
    return ne * vbar_cm_s(kT) / kT * exp(-t.P[Z] / kT) * lotz_shells(kT, t, Z, glx, glw);
}

__device__ inline double ln_rate_exact(double kT, double ne, const IonTables& t, int Z, const double* glx,
                                       const double* glw)
{
    if (!(kT > 0.0) || !(ne > 0.0)) return -INFINITY;
    return log(ne * vbar_cm_s(kT) / kT) - t.P[Z] / kT + log(lotz_shells(kT, t, Z, glx, glw));
}

}  // namespace pic
