// HIP kernels (gfx950) of the theta-grid path: one right-hand-side evaluation
// of the DMFE per RK stage, the RK stage combinations with the 1-norm error,
// and the sparsification residual.
//
// Data layout in HBM:
//   history  HPoint[M_cap][L]  slot-major; (C, R, dC/dt, dR/dt) of one
//            (t_n, theta_i) point are 32 contiguous bytes, so an s-point
//            stencil on one slice is s*32 contiguous bytes
//   slices   YPoint[L]         stage slices, RK stage derivatives, state
//   t_n, slot of slice n       logical order (slot indirection: sparsify and
//                              revert never move slice data)
#include <cmath>

#include "dmfe_internal.h"

namespace dmfe {
namespace {

constexpr int kWave = 64;

// ---------------------------------------------------------------- model polynomials
template <int NC>
__device__ __forceinline__ double horner(const double (&c)[PCAP], double q) {
    double acc = c[NC - 1];
#pragma unroll
    for (int k = NC - 2; k >= 0; --k) acc = fma(acc, q, c[k]);
    return acc;
}
// PM is the largest p the instantiation supports (f has PM+1 coefficients).
template <int PM> __device__ __forceinline__ double fF(const Model& m, double q) { return horner<PM + 1>(m.fc, q); }
template <int PM> __device__ __forceinline__ double fD1(const Model& m, double q) { return horner<PM>(m.f1, q); }
template <int PM> __device__ __forceinline__ double fD2(const Model& m, double q) { return horner<PM - 1>(m.f2, q); }

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}
// Sum over a block of up to 1024 threads; result valid in every thread.
// `sh` must hold 16 doubles; the call begins and ends with a barrier.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    __syncthreads();
    v = wave_sum(v);
    const int w = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    for (int q = 0; q < nw; ++q) r += sh[q];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- theta index map
// Continuous 0-based index of theta on the grid (inverse of eq. theta at
// alpha = 0): x = (L-1)/(2g) [log1p(e^g T) - log1p(-e^{-g} T)], T = tan(theta D)
// for theta <= 1/2; x = L-1 - x(1-theta) above, with the complement passed in.
__device__ __forceinline__ double xmap(const StageArgs& a, double th, double thc) {
    const bool lower = th <= 0.5;
    const double arg = lower ? th : thc;
    const double T = tan(arg * a.Dg);
    const double x = a.xscale * (log1p(a.eg * T) - log1p(-a.egi * T));
    return lower ? x : double(a.L - 1) - x;
}

// ---------------------------------------------------------------- index Lagrange stencil
__host__ __device__ constexpr double fact(int n) { return n <= 1 ? 1.0 : double(n) * fact(n - 1); }
__host__ __device__ constexpr double inv_den(int S, int k) {
    return (((S - 1 - k) & 1) ? -1.0 : 1.0) / (fact(k) * fact(S - 1 - k));
}
// Weights of the S-point Lagrange interpolant in the index coordinate on nodes
// base..base+S-1, base = floor(x) - (S-1)/2 clamped to [0, L-S].
template <int S>
__device__ __forceinline__ int lagrange(double x, int L, double (&w)[S]) {
    int base = int(floor(x)) - (S - 1) / 2;
    base = base < 0 ? 0 : (base > L - S ? L - S : base);
    const double u = x - double(base);
    double pre[S];
    double acc = 1.0;
#pragma unroll
    for (int k = 0; k < S; ++k) {
        pre[k] = acc;
        acc *= (u - double(k));
    }
    acc = 1.0;
#pragma unroll
    for (int k = S - 1; k >= 0; --k) {
        w[k] = pre[k] * acc * inv_den(S, k);
        acc *= (u - double(k));
    }
    return base;
}

template <int S>
__device__ __forceinline__ void interp2(const YPoint* row, int base, const double (&w)[S], double& c, double& r) {
    c = 0.0;
    r = 0.0;
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const YPoint v = row[base + k];
        c = fma(w[k], v.c, c);
        r = fma(w[k], v.r, r);
    }
}
template <int S>
__device__ __forceinline__ void interp4(const HPoint* row, int base, const double (&w)[S], HPoint& o) {
    o.c = o.r = o.dc = o.dr = 0.0;
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const HPoint v = row[base + k];
        o.c = fma(w[k], v.c, o.c);
        o.r = fma(w[k], v.r, o.r);
        o.dc = fma(w[k], v.dc, o.dc);
        o.dr = fma(w[k], v.dr, o.dr);
    }
}
template <int S>
__device__ __forceinline__ void interp2h(const HPoint* row, int base, const double (&w)[S], double& c, double& r) {
    c = 0.0;
    r = 0.0;
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const HPoint v = row[base + k];
        c = fma(w[k], v.c, c);
        r = fma(w[k], v.r, r);
    }
}

// largest m in [lo, hi-1] with t[m] <= x, given t[lo] <= x <= t[hi]
__device__ __forceinline__ int bracket(const double* t, int lo, int hi, double x) {
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (t[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------- stage prep: mu(t), E(t)
// mu(t) = T + t sum_i nu_i [f''(C)RC + f'(C)R]_i + beta0 f'(C_0) C_0 and
// E(t) = -t sum_i nu_i f'(C_i) R_i - beta0 f(C_0) on the stage slice (Sec. 2.1).
template <int PM>
__global__ __launch_bounds__(1024) void k_stage_prep(const Model m, int L, double t, const double* __restrict__ nu,
                                                     const YPoint* __restrict__ y, double* __restrict__ mue) {
    __shared__ double sh[16];
    double sk = 0.0, se = 0.0;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        const YPoint v = y[i];
        const double d1 = fD1<PM>(m, v.c), d2 = fD2<PM>(m, v.c);
        sk = fma(nu[i], d2 * v.r * v.c + d1 * v.r, sk);
        se = fma(nu[i], d1 * v.r, se);
    }
    sk = block_sum(sk, sh);
    se = block_sum(se, sh);
    if (threadIdx.x == 0) {
        const YPoint v0 = y[0];
        mue[0] = m.T + t * sk + m.beta0 * fD1<PM>(m, v0.c) * v0.c;
        mue[1] = -t * se - m.beta0 * fF<PM>(m, v0.c);
    }
}

// ---------------------------------------------------------------- the history integrals
// One wavefront per row j (t' = theta_j t); lanes walk the quadrature nodes i.
// Per pair (i, j) the kernel forms
//   a = (C,R)(t, theta_i theta_j t)        index Lagrange on the stage slice
//   b = (C,R)(t, phi t)                    phi = theta_j + (1-theta_j) theta_i
//   c = (C,R)(t', theta_i t')              Hermite in t on the row's bracket
//   d = (C,R)(phi t, psi phi t)            psi = theta_j/phi: Lagrange on the two
//                                          bracketing slices, then Hermite in t
// (targets inside the current step use the quadratic through value and d/dt of
// the last slice with a stored derivative and the stage slice), and the nine
// nu-weighted row sums of the forward, transposed and dual equations; lane 0
// assembles d/dt C(t, theta_j t) = d1C + theta_j d2C and likewise for R.
template <int S, int PM>
__global__ __launch_bounds__(256) void k_hist_integral(const StageArgs a) {
    extern __shared__ double s_t[];
    const int nb = a.nb;
    for (int q = threadIdx.x; q < nb; q += blockDim.x) s_t[q] = a.thist[q];
    __syncthreads();

    const int lane = threadIdx.x & (kWave - 1);
    const int j = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (j >= a.L) return;
    const int L = a.L;
    const double t = a.t, thj = a.th[j], thcj = a.thc[j], tp = thj * t;
    const int b = nb - 1;
    const double tb = a.tb;

    // row bracket for the c family (wave-uniform)
    int cmode;  // 0: stage slice only (t = 0), 1: slice 0, 2: Hermite, 3: in-step quadratic
    const HPoint* c0p = nullptr;
    const HPoint* c1p = nullptr;
    double cw0 = 0.0, cw1 = 0.0, cw2 = 0.0, cw3 = 0.0;
    if (nb == 0) {
        cmode = 0;
    } else if (tp <= tb) {
        if (b == 0) {
            cmode = 1;
            c0p = a.hist + size_t(a.slot[0]) * L;
        } else {
            cmode = 2;
            const int m = bracket(s_t, 0, b, tp);
            const double h = s_t[m + 1] - s_t[m];
            const double u = (tp - s_t[m]) / h;
            cw0 = 2 * u * u * u - 3 * u * u + 1;
            cw1 = (u * u * u - 2 * u * u + u) * h;
            cw2 = -2 * u * u * u + 3 * u * u;
            cw3 = (u * u * u - u * u) * h;
            c0p = a.hist + size_t(a.slot[m]) * L;
            c1p = a.hist + size_t(a.slot[m + 1]) * L;
        }
    } else {
        cmode = 3;
        const double h = t - tb;
        const double u = (tp - tb) / h;
        cw0 = 1.0 - u * u;
        cw1 = h * (u - u * u);
        cw2 = u * u;
        c0p = a.hist + size_t(a.slot[b]) * L;
    }
    const HPoint* bslot = nb >= 1 ? a.hist + size_t(a.slot[b]) * L : nullptr;
    const HPoint* slot0 = nb >= 1 ? a.hist + size_t(a.slot[0]) * L : nullptr;
    const double hq = t - tb;

    double S1 = 0, S2 = 0, S3 = 0, S4 = 0, S5 = 0, S6 = 0, S7 = 0, S8 = 0, S9 = 0;
    double c0C = 0.0;
    int lo = 0;
    for (int i = lane; i < L; i += kWave) {
        const double thi = a.th[i], thci = a.thc[i], w = a.nu[i];
        double wl[S];
        // a: (t, theta_i theta_j)
        double aC, aR;
        {
            const double x = xmap(a, thi * thj, fma(thi, thcj, thci));
            const int base = lagrange<S>(x, L, wl);
            interp2<S>(a.y, base, wl, aC, aR);
        }
        // b: (t, phi)
        const double phi = fma(thcj, thi, thj), phic = thcj * thci;
        double bC, bR;
        {
            const double x = xmap(a, phi, phic);
            const int base = lagrange<S>(x, L, wl);
            interp2<S>(a.y, base, wl, bC, bR);
        }
        // c: (t', theta_i)
        double cC, cR;
        if (cmode == 0) {
            const YPoint v = a.y[i];
            cC = v.c;
            cR = v.r;
        } else if (cmode == 1) {
            const HPoint v = c0p[i];
            cC = v.c;
            cR = v.r;
        } else if (cmode == 2) {
            const HPoint v0 = c0p[i], v1 = c1p[i];
            cC = cw0 * v0.c + cw1 * v0.dc + cw2 * v1.c + cw3 * v1.dc;
            cR = cw0 * v0.r + cw1 * v0.dr + cw2 * v1.r + cw3 * v1.dr;
        } else {
            const HPoint v0 = c0p[i];
            const YPoint yc = a.y[i];
            cC = cw0 * v0.c + cw1 * v0.dc + cw2 * yc.c;
            cR = cw0 * v0.r + cw1 * v0.dr + cw2 * yc.r;
        }
        if (i == 0) c0C = cC;
        // d: (phi t, psi)
        double dC, dR;
        {
            double psi = 0.0, psic = 1.0;  // psi = 0/0 := 0 at i = j = 0
            if (phi > 0.0) {
                psi = thj / phi;
                psic = thcj * thi / phi;
            }
            const double x = xmap(a, psi, psic);
            const int base = lagrange<S>(x, L, wl);
            const double s = phi * t;
            if (nb == 0) {
                interp2<S>(a.y, base, wl, dC, dR);
            } else if (s <= tb) {
                if (b == 0) {
                    interp2h<S>(slot0, base, wl, dC, dR);
                } else {
                    const int m = bracket(s_t, lo, b, s);
                    lo = m;
                    const double h = s_t[m + 1] - s_t[m];
                    const double u = (s - s_t[m]) / h;
                    HPoint p0, p1;
                    interp4<S>(a.hist + size_t(a.slot[m]) * L, base, wl, p0);
                    interp4<S>(a.hist + size_t(a.slot[m + 1]) * L, base, wl, p1);
                    const double h00 = 2 * u * u * u - 3 * u * u + 1, h10 = (u * u * u - 2 * u * u + u) * h;
                    const double h01 = -2 * u * u * u + 3 * u * u, h11 = (u * u * u - u * u) * h;
                    dC = h00 * p0.c + h10 * p0.dc + h01 * p1.c + h11 * p1.dc;
                    dR = h00 * p0.r + h10 * p0.dr + h01 * p1.r + h11 * p1.dr;
                }
            } else {
                HPoint pb;
                interp4<S>(bslot, base, wl, pb);
                double yc, yr;
                interp2<S>(a.y, base, wl, yc, yr);
                const double u = (s - tb) / hq;
                const double q0 = 1.0 - u * u, q1 = hq * (u - u * u), q2 = u * u;
                dC = q0 * pb.c + q1 * pb.dc + q2 * yc;
                dR = q0 * pb.r + q1 * pb.dr + q2 * yr;
            }
        }
        const double f2a = fD2<PM>(a.m, aC), f1a = fD1<PM>(a.m, aC);
        const double f2b = fD2<PM>(a.m, bC);
        const double f2c = fD2<PM>(a.m, cC), f1c = fD1<PM>(a.m, cC);
        const double f2d = fD2<PM>(a.m, dC), f1d = fD1<PM>(a.m, dC);
        S1 = fma(w, f2a * aR * cC, S1);
        S2 = fma(w, f1a * cR, S2);
        S3 = fma(w, f2b * bR * dC, S3);
        S4 = fma(w, f2b * bR * dR, S4);
        S5 = fma(w, f2c * cR * aC, S5);
        S6 = fma(w, f1c * aR, S6);
        S7 = fma(w, f1d * bR, S7);
        S8 = fma(w, bR * f2d * dR, S8);
        S9 = fma(w, f2c * cR * cC + f1c * cR, S9);
    }
    S1 = wave_sum(S1);
    S2 = wave_sum(S2);
    S3 = wave_sum(S3);
    S4 = wave_sum(S4);
    S5 = wave_sum(S5);
    S6 = wave_sum(S6);
    S7 = wave_sum(S7);
    S8 = wave_sum(S8);
    S9 = wave_sum(S9);
    if (lane == 0) {
        const double mu = a.mue[0];
        const YPoint y0 = a.y[0], yj = a.y[j];
        const double T = a.m.T, be = a.m.beta0;
        const double d1C = -mu * yj.c + t * (thj * S1 + thj * S2 + thcj * S3) + be * fD1<PM>(a.m, y0.c) * c0C;
        const double d1R = -mu * yj.r + t * thcj * S4;
        const double mup = T + t * thj * S9 + be * fD1<PM>(a.m, c0C) * c0C;
        const double d2C = -mup * yj.c + t * (thj * S5 + thj * S6 + thcj * S7) + 2.0 * T * yj.r +
                           be * fD1<PM>(a.m, c0C) * y0.c;
        const double d2R = mup * yj.r - t * thcj * S8;
        double oc = d1C + thj * d2C, orr = d1R + thj * d2R;
        if (j == L - 1) {
            a.diag[0] = oc;
            a.diag[1] = orr;
            oc = 0.0;
            orr = 0.0;
        }
        a.kout[j] = YPoint{oc, orr};
        if (a.store) {
            a.store[j].dc = oc;
            a.store[j].dr = orr;
        }
    }
}

// ---------------------------------------------------------------- RK stage combinations
struct Coef10 {
    double v[10];
};

// ys = y0 + dt sum_{l < nk} a_l k_l; the diagonal point is pinned to (1, 1).
__global__ void k_rk_combine(int L, const YPoint* __restrict__ y0, const YPoint* __restrict__ k, int nk,
                             const Coef10 a, double dt, YPoint* __restrict__ ys) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L) return;
    YPoint acc = y0[i];
    for (int l = 0; l < nk; ++l) {
        const double f = dt * a.v[l];
        const YPoint kv = k[size_t(l) * L + i];
        acc.c = fma(f, kv.c, acc.c);
        acc.r = fma(f, kv.r, acc.r);
    }
    if (i == L - 1) acc = YPoint{1.0, 1.0};
    ys[i] = acc;
}

// ynew = y0 + dt sum b_l k_l and eps = sum_i |dt sum e_l k_l| over both fields
// (Sec. 3.5), one block so that the sum has a fixed order.
__global__ __launch_bounds__(1024) void k_rk_finish(int L, const YPoint* __restrict__ y0,
                                                    const YPoint* __restrict__ k, int nk, const Coef10 bw,
                                                    const Coef10 ew, double dt, YPoint* __restrict__ ynew,
                                                    double* __restrict__ eps_out) {
    __shared__ double sh[16];
    double sum = 0.0;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        YPoint acc = y0[i];
        double ec = 0.0, er = 0.0;
        for (int l = 0; l < nk; ++l) {
            const YPoint kv = k[size_t(l) * L + i];
            const double f = dt * bw.v[l];
            acc.c = fma(f, kv.c, acc.c);
            acc.r = fma(f, kv.r, acc.r);
            ec = fma(ew.v[l], kv.c, ec);
            er = fma(ew.v[l], kv.r, er);
        }
        if (i == L - 1) acc = YPoint{1.0, 1.0};
        ynew[i] = acc;
        sum += fabs(dt * ec) + fabs(dt * er);
    }
    sum = block_sum(sum, sh);
    if (threadIdx.x == 0) eps_out[0] = sum;
}

__global__ void k_append(int L, const YPoint* __restrict__ y, HPoint* __restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L) return;
    dst[i].c = y[i].c;
    dst[i].r = y[i].r;
}

__global__ void k_load_state(int L, const HPoint* __restrict__ src, YPoint* __restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L) return;
    y[i] = YPoint{src[i].c, src[i].r};
}

// ---------------------------------------------------------------- sparsification residual
// eps_n = sum_i |Delta^C_n(theta_i)| + |Delta^R_n(theta_i)| with Delta the Hermite
// integral over [t_{n-1}, t_{n+1}] with slice n minus the one without (Sec. 3.6).
__device__ __forceinline__ double herm_int(double h, double ya, double da, double yb, double db) {
    return h * (ya + yb) * 0.5 + h * h * (da - db) * (1.0 / 12.0);
}
__global__ __launch_bounds__(256) void k_sparsify_residual(int L, int first, const double* __restrict__ thist,
                                                           const int* __restrict__ slot,
                                                           const HPoint* __restrict__ hist,
                                                           double* __restrict__ eps_n) {
    __shared__ double sh[16];
    const int n = first + blockIdx.x;
    const HPoint* pa = hist + size_t(slot[n - 1]) * L;
    const HPoint* pc = hist + size_t(slot[n]) * L;
    const HPoint* pb = hist + size_t(slot[n + 1]) * L;
    const double h1 = thist[n] - thist[n - 1], h2 = thist[n + 1] - thist[n], h3 = thist[n + 1] - thist[n - 1];
    double e = 0.0;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        const HPoint va = pa[i], vc = pc[i], vb = pb[i];
        const double dc = herm_int(h1, va.c, va.dc, vc.c, vc.dc) + herm_int(h2, vc.c, vc.dc, vb.c, vb.dc) -
                          herm_int(h3, va.c, va.dc, vb.c, vb.dc);
        const double dr = herm_int(h1, va.r, va.dr, vc.r, vc.dr) + herm_int(h2, vc.r, vc.dr, vb.r, vb.dr) -
                          herm_int(h3, va.r, va.dr, vb.r, vb.dr);
        e += fabs(dc) + fabs(dr);
    }
    e = block_sum(e, sh);
    if (threadIdx.x == 0) eps_n[n] = e;
}

// ---------------------------------------------------------------- observables and copies
template <int PM>
__global__ __launch_bounds__(256) void k_slice_observables(const Model m, int L, const double* __restrict__ nu,
                                                           const double* __restrict__ thist,
                                                           const int* __restrict__ slot,
                                                           const HPoint* __restrict__ hist, double* __restrict__ E,
                                                           double* __restrict__ mu) {
    __shared__ double sh[16];
    const int n = blockIdx.x;
    const HPoint* p = hist + size_t(slot[n]) * L;
    double sk = 0.0, se = 0.0;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        const HPoint v = p[i];
        const double d1 = fD1<PM>(m, v.c), d2 = fD2<PM>(m, v.c);
        sk = fma(nu[i], d2 * v.r * v.c + d1 * v.r, sk);
        se = fma(nu[i], d1 * v.r, se);
    }
    sk = block_sum(sk, sh);
    se = block_sum(se, sh);
    if (threadIdx.x == 0) {
        const double t = thist[n];
        const double c0 = p[0].c;
        if (mu) mu[n] = m.T + t * sk + m.beta0 * fD1<PM>(m, c0) * c0;
        if (E) E[n] = -t * se - m.beta0 * fF<PM>(m, c0);
    }
}

__global__ void k_pack(int L, int count, int field, const int* __restrict__ slot, const HPoint* __restrict__ hist,
                       double* __restrict__ dst) {
    const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= size_t(count) * L) return;
    const int n = int(idx / L), i = int(idx % L);
    const HPoint v = hist[size_t(slot[n]) * L + i];
    dst[idx] = field == 0 ? v.c : field == 1 ? v.r : field == 2 ? v.dc : v.dr;
}

__global__ void k_unpack(int L, int count, const double* __restrict__ C, const double* __restrict__ R,
                         const double* __restrict__ dC, const double* __restrict__ dR,
                         const int* __restrict__ slot, HPoint* __restrict__ hist) {
    const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= size_t(count) * L) return;
    const int n = int(idx / L), i = int(idx % L);
    hist[size_t(slot[n]) * L + i] = HPoint{C[idx], R[idx], dC[idx], dR[idx]};
}

__global__ void k_interleave(int L, const double* __restrict__ a, const double* __restrict__ b,
                             YPoint* __restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < L) y[i] = YPoint{a[i], b[i]};
}
__global__ void k_deinterleave(int L, const YPoint* __restrict__ y, double* __restrict__ a, double* __restrict__ b) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < L) {
        a[i] = y[i].c;
        b[i] = y[i].r;
    }
}

inline unsigned nblk(size_t n, unsigned bs) { return unsigned((n + bs - 1) / bs); }

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_stage_prep(const Model& m, int L, double t, const double* nu, const YPoint* y, double* mue,
                             hipStream_t st) {
    if (m.pmax <= 4) hipLaunchKernelGGL(k_stage_prep<4>, dim3(1), dim3(1024), 0, st, m, L, t, nu, y, mue);
    else hipLaunchKernelGGL(k_stage_prep<DMFE_MAX_P>, dim3(1), dim3(1024), 0, st, m, L, t, nu, y, mue);
    return hipGetLastError();
}

template <int S>
static hipError_t launch_hi_s(const StageArgs& a, hipStream_t st) {
    const unsigned rows_per_block = 4;
    const dim3 grid(nblk(a.L, rows_per_block)), block(rows_per_block * kWave);
    const size_t lds = size_t(a.nb > 0 ? a.nb : 1) * sizeof(double);
    if (a.m.pmax <= 4) hipLaunchKernelGGL((k_hist_integral<S, 4>), grid, block, lds, st, a);
    else hipLaunchKernelGGL((k_hist_integral<S, DMFE_MAX_P>), grid, block, lds, st, a);
    return hipGetLastError();
}

hipError_t launch_hist_integral(const StageArgs& a, int s, hipStream_t st) {
    switch (s) {
    case 4: return launch_hi_s<4>(a, st);
    case 6: return launch_hi_s<6>(a, st);
    case 8: return launch_hi_s<8>(a, st);
    case 10: return launch_hi_s<10>(a, st);
    case 12: return launch_hi_s<12>(a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_rk_combine(int L, const YPoint* y0, const YPoint* k, int nk, const double* coef, double dt,
                             YPoint* ys, hipStream_t st) {
    Coef10 a{};
    for (int l = 0; l < nk && l < 10; ++l) a.v[l] = coef[l];
    hipLaunchKernelGGL(k_rk_combine, dim3(nblk(L, 256)), dim3(256), 0, st, L, y0, k, nk, a, dt, ys);
    return hipGetLastError();
}

hipError_t launch_rk_finish(int L, const YPoint* y0, const YPoint* k, int nk, const double* b, const double* e,
                            double dt, YPoint* ynew, double* eps_out, hipStream_t st) {
    Coef10 bw{}, ew{};
    for (int l = 0; l < nk && l < 10; ++l) {
        bw.v[l] = b[l];
        ew.v[l] = e[l];
    }
    hipLaunchKernelGGL(k_rk_finish, dim3(1), dim3(1024), 0, st, L, y0, k, nk, bw, ew, dt, ynew, eps_out);
    return hipGetLastError();
}

hipError_t launch_append(int L, const YPoint* y, HPoint* slot_dst, hipStream_t st) {
    hipLaunchKernelGGL(k_append, dim3(nblk(L, 256)), dim3(256), 0, st, L, y, slot_dst);
    return hipGetLastError();
}

hipError_t launch_load_state(int L, const HPoint* slot_src, YPoint* y, hipStream_t st) {
    hipLaunchKernelGGL(k_load_state, dim3(nblk(L, 256)), dim3(256), 0, st, L, slot_src, y);
    return hipGetLastError();
}

hipError_t launch_sparsify_residual(int L, int first, int count, const double* thist, const int* slot,
                                    const HPoint* hist, double* eps_n, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sparsify_residual, dim3(count), dim3(256), 0, st, L, first, thist, slot, hist, eps_n);
    return hipGetLastError();
}

hipError_t launch_slice_observables(const Model& m, int L, const double* nu, int count, const double* thist,
                                    const int* slot, const HPoint* hist, double* E, double* mu, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    if (m.pmax <= 4)
        hipLaunchKernelGGL(k_slice_observables<4>, dim3(count), dim3(256), 0, st, m, L, nu, thist, slot, hist, E, mu);
    else
        hipLaunchKernelGGL(k_slice_observables<DMFE_MAX_P>, dim3(count), dim3(256), 0, st, m, L, nu, thist, slot,
                           hist, E, mu);
    return hipGetLastError();
}

hipError_t launch_pack_history(int L, int count, int field, const int* slot, const HPoint* hist, double* dst,
                               hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack, dim3(nblk(size_t(count) * L, 256)), dim3(256), 0, st, L, count, field, slot, hist,
                       dst);
    return hipGetLastError();
}

hipError_t launch_unpack_history(int L, int count, const double* C, const double* R, const double* dC,
                                 const double* dR, const int* slot, HPoint* hist, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpack, dim3(nblk(size_t(count) * L, 256)), dim3(256), 0, st, L, count, C, R, dC, dR, slot,
                       hist);
    return hipGetLastError();
}

hipError_t launch_interleave(int L, const double* a, const double* b, YPoint* y, hipStream_t st) {
    hipLaunchKernelGGL(k_interleave, dim3(nblk(L, 256)), dim3(256), 0, st, L, a, b, y);
    return hipGetLastError();
}

hipError_t launch_deinterleave(int L, const YPoint* y, double* a, double* b, hipStream_t st) {
    hipLaunchKernelGGL(k_deinterleave, dim3(nblk(L, 256)), dim3(256), 0, st, L, y, a, b);
    return hipGetLastError();
}

}  // namespace dmfe
