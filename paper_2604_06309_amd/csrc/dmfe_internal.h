// Internal declarations shared by the host core (api.hip) and the kernels
// (kernels_theta.hip, kernels_uniform.hip).  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/dmfe.h"

namespace dmfe {

// ---------------------------------------------------------------- host precompute (grid.cpp)
double lambert_gamma(double tmax);
void theta_grid(int L, double gamma, double* th, double* thc);
int quintic_weights(int L, const double* th, double* nu);
// rows b = 0..L-s of s barycentric coefficients and the inverse stencil span
void stencil_coefficients(int L, int s, int scheme, int d, const double* th, const double* thc, double* out);

// ---------------------------------------------------------------- model on the device
// f(q) = sum_k fc[k] q^k, f'(q) = sum_k f1[k] q^k, f''(q) = sum_k f2[k] q^k with
// zero-padded dense coefficients (k < PCAP), evaluated by Horner.
constexpr int PCAP = DMFE_MAX_P + 1;
struct Model {
    double T, beta0;
    double fc[PCAP];
    double f1[PCAP];
    double f2[PCAP];
    int pmax;  // largest p in the mixture
};

// One history point in HBM: the four stored fields at (t_n, theta_i).
struct alignas(32) HPoint {
    double c, r, dc, dr;
};
// The same point stored in single precision (DMFE_FP32_COMP histories).
struct alignas(16) HPoint32 {
    float c, r, dc, dr;
};
// One point of a stage slice (the RK state vector is interleaved C, R).
struct alignas(16) YPoint {
    double c, r;
};

// log-R option (Appendix A): log R and the scaled derivative (dR/dt)/R of one
// stored point, computed once per point from the stored values; NaN where R <= 0,
// so that a stencil holding such a point falls back to R itself.
struct alignas(16) LogPoint {
    double lr, lg;
};

// Arguments of one right-hand-side evaluation on the theta grid.
struct StageArgs {
    int L;
    int nb;              // slices 0..nb-1 carry valid d/dt
    double t;            // stage time
    double tb;           // t of slice nb-1 (unused when nb == 0)
    const double* X;     // X[j][i] = x(theta_i theta_j), continuous grid index [L][L]
    const double* Xd;    // Xd[j][i] = x(psi_ij), psi = theta_j / phi_ij [L][L]
    const double* th;    // theta_i [L]
    const double* thc;   // 1 - theta_i [L]
    const double* nu;    // quadrature weights [L]
    const double* thist; // t_n in logical order [>= nb]
    const int* slot;     // slot of logical slice n [>= nb]
    const void* hist;    // history slots [M_cap][L] of HPoint (fp64) or HPoint32 (fp32 histories)
    const void* stage;   // the stage slice in history format [L] (written by the stage prep)
    const YPoint* y;     // stage slice [L]
    const double* mue;   // mu(t), E(t) of the stage slice [2]
    YPoint* kout;        // d/dt C, d/dt R along fixed theta [L]
    void* store;         // if not null: slot whose dc, dr receive kout (row L-1 stored as 0)
    int fp32;            // history precision: 0 = HPoint, 1 = HPoint32
    double* diag;        // computed values of row L-1 [2]
    Model m;
    int interp;          // DMFE_INTERP_* scheme in theta
    int log_r;           // interpolate log R (falls back to R on non-positive stencils)
    const double* bw;    // barycentric stencil coefficients [L-s+1][s+1] (schemes other than index Lagrange)
    double fh_c[16];     // index Floater-Hormann: the coefficients, the same for every stencil base
    LogPoint* lhist;     // log-R option: log mirror of the history slots [M_cap][L], else null
    const LogPoint* lstage;  // log-R option: log mirror of the stage slot [L], else null
};

// Run-constant data of the theta grid used by the coordinate precompute.
struct GridArgs {
    int L;
    double xscale;  // (L-1) / (2 gamma)
    double eg, egi; // e^gamma, e^{-gamma}
    double Dg;      // atan(sinh gamma)
    const double* th;
    const double* thc;
    double* X;
    double* Xd;
};

// launchers (kernels_theta.hip); all return hipError_t of the launch
hipError_t launch_coords(const GridArgs& g, hipStream_t st);
hipError_t launch_stage_prep(const Model& m, int L, double t, const double* nu, const YPoint* y, double* mue,
                             void* stage, int fp32, LogPoint* lstage, hipStream_t st);
hipError_t launch_hist_integral(const StageArgs& a, int s, hipStream_t st);
hipError_t launch_rk_combine(int L, const YPoint* y0, const YPoint* k, int nk, const double* coef, double dt,
                             YPoint* ys, hipStream_t st);
hipError_t launch_rk_finish(int L, const YPoint* y0, const YPoint* k, int nk, const double* b, const double* e,
                            double dt, YPoint* ynew, double* eps_out, hipStream_t st);
// History pointers below are HPoint* when fp32 == 0 and HPoint32* when fp32 == 1.
// Accepting a step: y_new into slot_dst (as (C, R)) and into y0; k_last -> k_first when
// k_first is set (first-same-as-last); t_new and slot_new at index M of the device
// time and slot arrays; the slot's log mirror when lslot is set.
struct AcceptArgs {
    int L, M, slot_new;
    double t_new;
    const YPoint* ynew;
    void* slot_dst;
    LogPoint* lslot;
    YPoint* y0;
    const YPoint* k_last;
    YPoint* k_first;
    double* thist;
    int* slots;
};
hipError_t launch_accept(const AcceptArgs& a, int fp32, hipStream_t st);
// the log mirror of `count` stored slices (log-R option) from their stored values
hipError_t launch_log_mirror(int L, int count, const int* slot, const void* hist, int fp32, LogPoint* lhist,
                             hipStream_t st);
hipError_t launch_load_state(int L, const void* slot_src, int fp32, YPoint* y, hipStream_t st);
// part: scratch of 2 * sparsify_chunks(L) * stride doubles (stride >= first + count + 1)
int sparsify_chunks(int L);
hipError_t launch_sparsify_residual(int L, int first, int count, const double* thist, const int* slot,
                                    const void* hist, int fp32, double* eps_n, double* part, int stride,
                                    hipStream_t st);
hipError_t launch_slice_observables(const Model& m, int L, const double* nu, int count, const double* thist,
                                    const int* slot, const void* hist, int fp32, double* E, double* mu,
                                    hipStream_t st);
hipError_t launch_pack_history(int L, int count, int field, const int* slot, const void* hist, int fp32,
                               double* dst, hipStream_t st);
hipError_t launch_unpack_history(int L, int count, const double* C, const double* R, const double* dC,
                                 const double* dR, const int* slot, void* hist, int fp32, hipStream_t st);
hipError_t launch_interleave(int L, const double* a, const double* b, YPoint* y, hipStream_t st);
hipError_t launch_deinterleave(int L, const YPoint* y, double* a, double* b, hipStream_t st);

// ---------------------------------------------------------------- many instances per launch (serving)
// Block b of a batched launch belongs to instance q with first_block[q] <= b < first_block[q+1].
struct CombineDesc {
    const YPoint* y0;
    const YPoint* k;
    YPoint* ys;
    int L, nk;
    double dt;
    double a[10];
};
struct PrepDesc {
    const YPoint* y;
    const double* nu;
    double* mue;
    void* stage;  // the stage slice in history format [L]
    int L;
    int fp32;
    double t;
    Model m;
};
struct FinishDesc {
    const YPoint* y0;
    const YPoint* k;
    YPoint* ynew;
    double* eps;
    int L, nk;
    double dt;
    double b[10], e[10];
};
hipError_t launch_rk_combine_multi(const CombineDesc* d, const int* first_block, int n, int total_blocks,
                                   hipStream_t st);
hipError_t launch_stage_prep_multi(const PrepDesc* d, int n, int pmax, hipStream_t st);
hipError_t launch_hist_integral_multi(const StageArgs* d, const int* first_block, int n, int total_blocks, int s,
                                      int pmax, int fp32, int nb_max, hipStream_t st);
hipError_t launch_rk_finish_multi(const FinishDesc* d, int n, hipStream_t st);
constexpr int kCombineBlock = 256;
// Rows of the theta grid per history-integral block: 4 with an FP64 history, 8 with FP32.
constexpr int hist_rows_per_block(int fp32) { return fp32 ? 8 : 4; }

// ---------------------------------------------------------------- uniform mode (kernels_uniform.hip)
struct UniArgs {
    int n;          // current row: unknowns k = 0..n
    double h;       // grid step
    double delta;   // stage offset t - t_n
    const double* C;  // packed lower triangle, rows 0..n
    const double* R;
    const double* y;  // stage unknowns: c_k = y[k], r_k = y[cap + k]
    int cap;          // stride between the c and r halves of y / kout
    double* kout;
    Model m;
};
hipError_t launch_uniform_rhs(const UniArgs& a, hipStream_t st);
hipError_t launch_uniform_axpy(int n1, int cap, const double* y0, const double* k, double a, double* out,
                               hipStream_t st);
hipError_t launch_uniform_rk4_append(int n, int cap, double h, const double* y0, const double* k1,
                                     const double* k2, const double* k3, const double* k4, double* C, double* R,
                                     double* y_next, hipStream_t st);
hipError_t launch_uniform_energy(const Model& m, int n, double h, const double* C, const double* R, double* E,
                                 hipStream_t st);

}  // namespace dmfe
