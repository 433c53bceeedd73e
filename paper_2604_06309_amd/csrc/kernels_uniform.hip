// HIP kernels (gfx950) of the uniform-grid path: C(t_n, t_k), R(t_n, t_k) on an
// equidistant grid, classical RK4 in t, trapezoid history integrals with the
// partial panel [t_n, t] closed by the diagonal values C(t,t) = R(t,t^-) = 1.
//
// Storage: packed lower triangles, row n = X[n][0..n] at offset n(n+1)/2.
// Stage unknowns y = (c_0..c_n | r_0..r_n) with the r half at offset `cap`.
#include <cmath>

#include "dmfe_internal.h"

namespace dmfe {
namespace {

constexpr int kWave = 64;

template <int NC>
__device__ __forceinline__ double horner(const double (&c)[PCAP], double q) {
    double acc = c[NC - 1];
#pragma unroll
    for (int k = NC - 2; k >= 0; --k) acc = fma(acc, q, c[k]);
    return acc;
}
template <int PM> __device__ __forceinline__ double fF(const Model& m, double q) { return horner<PM + 1>(m.fc, q); }
template <int PM> __device__ __forceinline__ double fD1(const Model& m, double q) { return horner<PM>(m.f1, q); }
template <int PM> __device__ __forceinline__ double fD2(const Model& m, double q) { return horner<PM - 1>(m.f2, q); }

__device__ __forceinline__ size_t tri(int n, int k) { return size_t(n) * (n + 1) / 2 + k; }

// trapezoid weight of node q on nodes lo..hi with spacing h (0 when lo == hi)
__device__ __forceinline__ double trap(int q, int lo, int hi, double h) {
    if (hi <= lo) return 0.0;
    return (q == lo || q == hi) ? 0.5 * h : h;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// One block per k = 0..n: the integrals
//   A_k = int_0^t K(t,s) C(s,t_k) ds,  B_k = int_0^{t_k} D(t,s) R(t_k,s) ds,
//   Q_k = int_{t_k}^t K(t,s) R(s,t_k) ds,  and mu(t),
// then dc_k = -mu c_k + A_k + B_k + beta0 f'(c_0) C(t_k,0), dr_k = -mu r_k + Q_k.
template <int PM>
__global__ __launch_bounds__(256) void k_uniform_rhs(const UniArgs a) {
    __shared__ double sh[4][4];
    const int k = blockIdx.x, n = a.n, cap = a.cap;
    const double h = a.h, delta = a.delta;
    const double* c = a.y;
    const double* r = a.y + cap;
    double smu = 0.0, sA = 0.0, sB = 0.0, sQ = 0.0;
    for (int q = threadIdx.x; q <= n; q += blockDim.x) {
        const double cq = c[q], rq = r[q];
        const double f2 = fD2<PM>(a.m, cq), f1 = fD1<PM>(a.m, cq);
        const double W = trap(q, 0, n, h) + (q == n ? 0.5 * delta : 0.0);
        smu = fma(W, f2 * rq * cq + f1 * rq, smu);
        const double Cqk = q >= k ? a.C[tri(q, k)] : a.C[tri(k, q)];
        sA = fma(W, f2 * rq * Cqk, sA);
        if (q <= k) sB = fma(trap(q, 0, k, h), f1 * a.R[tri(k, q)], sB);
        if (q >= k) {
            const double U = trap(q, k, n, h) + (q == n ? 0.5 * delta : 0.0);
            sQ = fma(U, f2 * rq * a.R[tri(q, k)], sQ);
        }
    }
    smu = wave_sum(smu);
    sA = wave_sum(sA);
    sB = wave_sum(sB);
    sQ = wave_sum(sQ);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        sh[w][0] = smu;
        sh[w][1] = sA;
        sh[w][2] = sB;
        sh[w][3] = sQ;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tmu = 0, tA = 0, tB = 0, tQ = 0;
        for (int q = 0; q < int(blockDim.x / kWave); ++q) {
            tmu += sh[q][0];
            tA += sh[q][1];
            tB += sh[q][2];
            tQ += sh[q][3];
        }
        const double Ws = 0.5 * delta;
        const double f1one = fD1<PM>(a.m, 1.0), f2one = fD2<PM>(a.m, 1.0);
        const double mu = a.m.T + tmu + Ws * (f2one + f1one) + a.m.beta0 * fD1<PM>(a.m, c[0]) * c[0];
        const double A = tA + Ws * f2one * c[k];
        const double Q = tQ + Ws * f2one * r[k];
        a.kout[k] = -mu * c[k] + A + tB + a.m.beta0 * fD1<PM>(a.m, c[0]) * a.C[tri(k, 0)];
        a.kout[cap + k] = -mu * r[k] + Q;
    }
}

__global__ void k_uniform_axpy(int n1, int cap, const double* __restrict__ y0, const double* __restrict__ k,
                               double s, double* __restrict__ out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n1) return;
    out[q] = y0[q] + s * k[q];
    out[cap + q] = y0[cap + q] + s * k[cap + q];
}

// row n+1 of the triangles from the RK4 combination; the diagonal is 1
__global__ void k_uniform_rk4_append(int n, int cap, double h, const double* __restrict__ y0,
                                     const double* __restrict__ k1, const double* __restrict__ k2,
                                     const double* __restrict__ k3, const double* __restrict__ k4,
                                     double* __restrict__ C, double* __restrict__ R, double* __restrict__ ynext) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q > n + 1) return;
    if (q == n + 1) {
        C[tri(n + 1, n + 1)] = 1.0;
        R[tri(n + 1, n + 1)] = 1.0;
        ynext[q] = 1.0;
        ynext[cap + q] = 1.0;
        return;
    }
    const double cn = y0[q] + h / 6.0 * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
    const int p = cap + q;
    const double rn = y0[p] + h / 6.0 * (k1[p] + 2.0 * k2[p] + 2.0 * k3[p] + k4[p]);
    C[tri(n + 1, q)] = cn;
    R[tri(n + 1, q)] = rn;
    ynext[q] = cn;
    ynext[p] = rn;
}

// E(t_n) = -int_0^{t_n} f'(C(t_n,s)) R(t_n,s) ds - beta0 f(C(t_n,0))
template <int PM>
__global__ __launch_bounds__(256) void k_uniform_energy(const Model m, int n, double h, const double* __restrict__ C,
                                                        const double* __restrict__ R, double* __restrict__ E) {
    __shared__ double sh[4];
    double s = 0.0;
    for (int q = threadIdx.x; q <= n; q += blockDim.x)
        s = fma(trap(q, 0, n, h), fD1<PM>(m, C[tri(n, q)]) * R[tri(n, q)], s);
    s = wave_sum(s);
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int q = 0; q < int(blockDim.x / kWave); ++q) tot += sh[q];
        E[n] = -tot - m.beta0 * fF<PM>(m, C[tri(n, 0)]);
    }
}

inline unsigned nblk(size_t n, unsigned bs) { return unsigned((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_uniform_rhs(const UniArgs& a, hipStream_t st) {
    if (a.m.pmax <= 4) hipLaunchKernelGGL(k_uniform_rhs<4>, dim3(a.n + 1), dim3(256), 0, st, a);
    else hipLaunchKernelGGL(k_uniform_rhs<DMFE_MAX_P>, dim3(a.n + 1), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_uniform_axpy(int n1, int cap, const double* y0, const double* k, double a, double* out,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_uniform_axpy, dim3(nblk(n1, 256)), dim3(256), 0, st, n1, cap, y0, k, a, out);
    return hipGetLastError();
}

hipError_t launch_uniform_rk4_append(int n, int cap, double h, const double* y0, const double* k1,
                                     const double* k2, const double* k3, const double* k4, double* C, double* R,
                                     double* y_next, hipStream_t st) {
    hipLaunchKernelGGL(k_uniform_rk4_append, dim3(nblk(n + 2, 256)), dim3(256), 0, st, n, cap, h, y0, k1, k2, k3, k4,
                       C, R, y_next);
    return hipGetLastError();
}

hipError_t launch_uniform_energy(const Model& m, int n, double h, const double* C, const double* R, double* E,
                                 hipStream_t st) {
    if (m.pmax <= 4) hipLaunchKernelGGL(k_uniform_energy<4>, dim3(1), dim3(256), 0, st, m, n, h, C, R, E);
    else hipLaunchKernelGGL(k_uniform_energy<DMFE_MAX_P>, dim3(1), dim3(256), 0, st, m, n, h, C, R, E);
    return hipGetLastError();
}

}  // namespace dmfe
