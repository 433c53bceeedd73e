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
// One point of a stage slice (the RK state vector is interleaved C, R).
struct alignas(16) YPoint {
    double c, r;
};

// Arguments of one right-hand-side evaluation on the theta grid.
struct StageArgs {
    int L;
    int nb;              // slices 0..nb-1 carry valid d/dt
    double t;            // stage time
    double tb;           // t of slice nb-1 (unused when nb == 0)
    double xscale;       // (L-1) / (2 gamma)
    double eg, egi;      // e^gamma, e^{-gamma}
    double Dg;           // atan(sinh gamma)
    const double* th;    // theta_i [L]
    const double* thc;   // 1 - theta_i [L]
    const double* nu;    // quadrature weights [L]
    const double* thist; // t_n in logical order [>= nb]
    const int* slot;     // slot of logical slice n [>= nb]
    const HPoint* hist;  // history slots [M_cap][L]
    const YPoint* y;     // stage slice [L]
    const double* mue;   // mu(t), E(t) of the stage slice [2]
    YPoint* kout;        // d/dt C, d/dt R along fixed theta [L]
    HPoint* store;       // if not null: slot whose dc, dr receive kout (row L-1 stored as 0)
    double* diag;        // computed values of row L-1 [2]
    Model m;
};

// launchers (kernels_theta.hip); all return hipError_t of the launch
hipError_t launch_stage_prep(const Model& m, int L, double t, const double* nu, const YPoint* y, double* mue,
                             hipStream_t st);
hipError_t launch_hist_integral(const StageArgs& a, int s, hipStream_t st);
hipError_t launch_rk_combine(int L, const YPoint* y0, const YPoint* k, int nk, const double* coef, double dt,
                             YPoint* ys, hipStream_t st);
hipError_t launch_rk_finish(int L, const YPoint* y0, const YPoint* k, int nk, const double* b, const double* e,
                            double dt, YPoint* ynew, double* eps_out, hipStream_t st);
hipError_t launch_append(int L, const YPoint* y, HPoint* slot_dst, hipStream_t st);
hipError_t launch_load_state(int L, const HPoint* slot_src, YPoint* y, hipStream_t st);
hipError_t launch_sparsify_residual(int L, int first, int count, const double* thist, const int* slot,
                                    const HPoint* hist, double* eps_n, hipStream_t st);
hipError_t launch_slice_observables(const Model& m, int L, const double* nu, int count, const double* thist,
                                    const int* slot, const HPoint* hist, double* E, double* mu, hipStream_t st);
hipError_t launch_pack_history(int L, int count, int field, const int* slot, const HPoint* hist, double* dst,
                               hipStream_t st);
hipError_t launch_unpack_history(int L, int count, const double* C, const double* R, const double* dC,
                                 const double* dR, const int* slot, HPoint* hist, hipStream_t st);
hipError_t launch_interleave(int L, const double* a, const double* b, YPoint* y, hipStream_t st);
hipError_t launch_deinterleave(int L, const YPoint* y, double* a, double* b, hipStream_t st);

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
