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
#include <map>
#include <mutex>
#include <utility>

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
__device__ __forceinline__ double xmap(const GridArgs& a, double th, double thc) {
    const bool lower = th <= 0.5;
    const double arg = lower ? th : thc;
    const double T = tan(arg * a.Dg);
    const double x = a.xscale * (log1p(a.eg * T) - log1p(-a.egi * T));
    return lower ? x : double(a.L - 1) - x;
}

// The interpolation coordinates depend only on the grid, so they are formed
// once per solver: X[j][i] = x(theta_i theta_j) (with its complement
// 1 - theta_i theta_j = (1-theta_i) + theta_i (1-theta_j)) and
// Xd[j][i] = x(psi_ij), psi = theta_j/phi, 1 - psi = (1-theta_j) theta_i/phi.
// Because theta_{L-1-i} = 1 - theta_i on this grid, x(phi_ij) =
// L-1 - X[L-1-j][L-1-i] and the phi family needs no table of its own.
__global__ void k_coords(const GridArgs g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= g.L) return;
    const double thi = g.th[i], thci = g.thc[i], thj = g.th[j], thcj = g.thc[j];
    g.X[size_t(j) * g.L + i] = xmap(g, thi * thj, fma(thi, thcj, thci));
    const double phi = fma(thcj, thi, thj);
    double psi = 0.0, psic = 1.0;  // psi = 0/0 := 0 at i = j = 0
    if (phi > 0.0) {
        psi = thj / phi;
        psic = thcj * thi / phi;
    }
    g.Xd[size_t(j) * g.L + i] = xmap(g, psi, psic);
}

// ---------------------------------------------------------------- index Lagrange stencil
// 1 / prod_{l != k} (k - l) = (-1)^(S-1-k) / (k! (S-1-k)!), as a compile-time table
template <int S>
struct InvDen {
    double v[S];
    constexpr InvDen() : v() {
        for (int k = 0; k < S; ++k) {
            double f = 1.0;
            for (int q = 2; q <= k; ++q) f *= q;
            for (int q = 2; q <= S - 1 - k; ++q) f *= q;
            v[k] = (((S - 1 - k) & 1) ? -1.0 : 1.0) / f;
        }
    }
};
// Weights of the S-point Lagrange interpolant in the index coordinate on nodes
// base..base+S-1, base = floor(x) - (S-1)/2 clamped to [0, L-S].
// The offset u = x - base is formed in double; the weights are computed in R.
template <int S, class R = double>
__device__ __forceinline__ int lagrange(double x, int L, R (&w)[S]) {
    int base = int(floor(x)) - (S - 1) / 2;
    base = base < 0 ? 0 : (base > L - S ? L - S : base);
    const R u = R(x - double(base));
    constexpr InvDen<S> den{};
    R pre[S];
    R acc = R(1);
#pragma unroll
    for (int k = 0; k < S; ++k) {
        pre[k] = acc;
        acc *= (u - R(k));
    }
    acc = R(1);
#pragma unroll
    for (int k = S - 1; k >= 0; --k) {
        w[k] = pre[k] * acc * R(den.v[k]);
        acc *= (u - R(k));
    }
    return base;
}

// Arithmetic type of values read from a history point type.
template <class HP> struct HReal;
template <> struct HReal<HPoint> { using type = double; };
template <> struct HReal<HPoint32> { using type = float; };
template <class HP> using hreal_t = typename HReal<HP>::type;

template <int S, int U = S>
__device__ __forceinline__ void interp2(const YPoint* row, int base, const double (&w)[S], double& c, double& r) {
    c = 0.0;
    r = 0.0;
#pragma unroll U
    for (int k = 0; k < S; ++k) {
        const YPoint v = row[base + k];
        c = fma(w[k], v.c, c);
        r = fma(w[k], v.r, r);
    }
}
// The same sums with all S reads issued before the first product (the scheduler
// otherwise waits on each read in turn); the sums are formed in the same order.
template <int S>
__device__ __forceinline__ void interp2_batched(const YPoint* row, int base, const double (&w)[S], double& c,
                                                double& r) {
    YPoint v[S];
#pragma unroll
    for (int k = 0; k < S; ++k) v[k] = row[base + k];
    __builtin_amdgcn_sched_barrier(0);
    c = 0.0;
    r = 0.0;
#pragma unroll
    for (int k = 0; k < S; ++k) {
        c = fma(w[k], v[k].c, c);
        r = fma(w[k], v[k].r, r);
    }
}
template <int S, class HP, class R = hreal_t<HP>>
__device__ __forceinline__ void interp4(const HP* row, int base, const R (&w)[S], R& c, R& r, R& dc, R& dr) {
    c = r = dc = dr = R(0);
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const HP v = row[base + k];
        c = fma(w[k], v.c, c);
        r = fma(w[k], v.r, r);
        dc = fma(w[k], v.dc, dc);
        dr = fma(w[k], v.dr, dr);
    }
}

// Nodes per slot of a wave's shared-node buffer (below): 28 keeps a block's LDS
// within 160 KB with the times of 16384 slices beside it.
constexpr int kTileNodes = 28;

// The 2-D stencil of one target on two slots, read in batches of 5 points of an FP64
// history (10 loads in flight per lane before the first product) or 10 of an FP32
// history (the same 40 registers; 5 for stencils above 14 points, whose registers
// would spill), values widened to FP64 as they are used, sums in the order of interp4.
template <int S, class HP>
__device__ __forceinline__ void gathered_stencil(const HP* p0, const HP* p1, int base, const double (&w)[S],
                                                 double& c0, double& r0, double& dc0, double& dr0, double& c1,
                                                 double& r1, double& dc1, double& dr1) {
    constexpr int B = sizeof(HP) == sizeof(HPoint) || S > 14 ? 5 : 10;
    c0 = r0 = dc0 = dr0 = c1 = r1 = dc1 = dr1 = 0.0;
#pragma unroll
    for (int kb = 0; kb < 2 * S; kb += B) {
        HP v[B];
#pragma unroll
        for (int q = 0; q < B; ++q) {
            const int k = kb + q;
            if (k < 2 * S) v[q] = k < S ? p0[base + k] : p1[base + k - S];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < B; ++q) {
            const int k = kb + q;
            if (k < S) {
                c0 = fma(w[k], double(v[q].c), c0);
                r0 = fma(w[k], double(v[q].r), r0);
                dc0 = fma(w[k], double(v[q].dc), dc0);
                dr0 = fma(w[k], double(v[q].dr), dr0);
            } else if (k < 2 * S) {
                c1 = fma(w[k - S], double(v[q].c), c1);
                r1 = fma(w[k - S], double(v[q].r), r1);
                dc1 = fma(w[k - S], double(v[q].dc), dc1);
                dr1 = fma(w[k - S], double(v[q].dr), dr1);
            }
        }
    }
}
// The same from a wave's LDS buffer: the first slot's nodes at [0, kTileNodes), the
// second's at [kTileNodes, 2 kTileNodes), this stencil at offset off in each.
template <int S, class LP>
__device__ __forceinline__ void shared_stencil(const LP* tile, int off, const double (&w)[S], double& c0,
                                               double& r0, double& dc0, double& dr0, double& c1, double& r1,
                                               double& dc1, double& dr1) {
    constexpr int B = 5;
    c0 = r0 = dc0 = dr0 = c1 = r1 = dc1 = dr1 = 0.0;
#pragma unroll
    for (int kb = 0; kb < 2 * S; kb += B) {
        double vc[B], vr[B], vdc[B], vdr[B];
#pragma unroll
        for (int q = 0; q < B; ++q) {
            const int k = kb + q;
            if (k < 2 * S) {
                const int id = k < S ? off + k : kTileNodes + off + k - S;
                vc[q] = tile[id].c;
                vr[q] = tile[id].r;
                vdc[q] = tile[id].dc;
                vdr[q] = tile[id].dr;
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < B; ++q) {
            const int k = kb + q;
            if (k < S) {
                c0 = fma(w[k], vc[q], c0);
                r0 = fma(w[k], vr[q], r0);
                dc0 = fma(w[k], vdc[q], dc0);
                dr0 = fma(w[k], vdr[q], dr0);
            } else if (k < 2 * S) {
                c1 = fma(w[k - S], vc[q], c1);
                r1 = fma(w[k - S], vr[q], r1);
                dc1 = fma(w[k - S], vdc[q], dc1);
                dr1 = fma(w[k - S], vdr[q], dr1);
            }
        }
    }
}

// ---------------------------------------------------------------- the other theta schemes
// Weights of the stencil of a target under the handle's scheme (Sec. 3.3); the
// target has continuous index x, theta tq and 1 - theta tqc.  Index Lagrange is
// the closed form above; the others use the barycentric form
//   w_k = c_k P_k / sum_m c_m P_m,  P_k = prod_{m != k} dz_m,
// with dz_m = u - m on the index coordinate (u = x - base) and the scaled theta
// differences (tq - theta_m) or ((1 - theta_m) - tqc) (tq above 1/2) on theta,
// and the coefficients c_k of the stencil's base from the host table.  At a node
// every P_k but one vanishes, so the weights are exact unit vectors there.
//
// Kernel variants: the default stencil (index Lagrange, R itself) and three for
// the other options, each compiled on its own so that no variant carries the
// registers of another.
enum : int { kVarDefault = 0, kVarIndexLagrangeLog = 1, kVarIndexFH = 2, kVarTheta = 3, kVarIndexFHLog = 4,
              kVarThetaLog = 5 };
constexpr bool var_log(int v) { return v == kVarIndexLagrangeLog || v == kVarIndexFHLog || v == kVarThetaLog; }
constexpr bool var_index_fh(int v) { return v == kVarIndexFH || v == kVarIndexFHLog; }
constexpr bool var_theta(int v) { return v == kVarTheta || v == kVarThetaLog; }
template <int S, int VAR>
__device__ __forceinline__ int stencil_weights(const StageArgs& a, double x, double tq, double tqc, double (&w)[S]) {
    if constexpr (VAR == kVarDefault || VAR == kVarIndexLagrangeLog) return lagrange<S>(x, a.L, w);
    int base = int(floor(x)) - (S - 1) / 2;
    base = base < 0 ? 0 : (base > a.L - S ? a.L - S : base);
    // on the index coordinate every stencil has the same coefficients (kernel arguments)
    const double* c = var_index_fh(VAR) ? a.fh_c : a.bw + size_t(base) * (S + 1);
    double dz[S];
    if constexpr (var_index_fh(VAR)) {
        const double u = x - double(base);
#pragma unroll
        for (int k = 0; k < S; ++k) dz[k] = u - double(k);
    } else {
        // theta below 1/2, the complement above: dz = +-(z - z_k) / span
        const bool lo = tq <= 0.5;
        const double* zn = lo ? a.th : a.thc;
        const double zt = lo ? tq : tqc;
        const double f = lo ? c[S] : -c[S];
#pragma unroll
        for (int k = 0; k < S; ++k) dz[k] = (zt - zn[base + k]) * f;
    }
    double pre[S];
    double acc = 1.0;
#pragma unroll
    for (int k = 0; k < S; ++k) {
        pre[k] = acc;
        acc *= dz[k];
    }
    acc = 1.0;
    double sum = 0.0;
#pragma unroll
    for (int k = S - 1; k >= 0; --k) {
        w[k] = c[k] * pre[k] * acc;
        acc *= dz[k];
        sum += w[k];
    }
    const double inv = 1.0 / sum;
#pragma unroll
    for (int k = 0; k < S; ++k) w[k] *= inv;
    return base;
}

// The log-R option (Appendix A) reads the log mirror: log R and (dR/dt)/R of every
// stored point, formed once when the point is stored (NaN where R <= 0).  A
// value is interpolated in log R with the same weights and exponentiated; a NaN
// in any point read (a non-positive R) leaves the plain value.
__device__ __forceinline__ LogPoint log_point(double r, double dr) {
    const double nan = __builtin_nan("");
    return r > 0.0 ? LogPoint{log(r), dr / r} : LogPoint{nan, nan};
}
template <int S>
__device__ __forceinline__ double log_interp_stage(const LogPoint* row, int base, const double (&w)[S], double plain) {
    double l = 0.0;
#pragma unroll
    for (int k = 0; k < S; ++k) l = fma(w[k], row[base + k].lr, l);
    return __builtin_isnan(l) ? plain : exp(l);
}
template <int S>
__device__ __forceinline__ void log_interp_slot(const LogPoint* row, int base, const double (&w)[S], double& lv,
                                                double& ld) {
    lv = 0.0;
    ld = 0.0;
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const LogPoint q = row[base + k];
        lv = fma(w[k], q.lr, lv);
        ld = fma(w[k], q.lg, ld);
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
// The same pass writes the stage slice into the stage slot in history format,
// so that targets inside the current step are gathered like stored ones: an
// FP64 slot holds (C, R, 0, 0); an FP32 slot holds the FP32 value and its
// rounding remainder (C_hi, R_hi, C - C_hi, R - R_hi), which a reader weighting
// both fields equally sums back to the FP64 value up to 2^-48.
__device__ __forceinline__ void write_stage_point(void* stage, int fp32, int i, const YPoint& v) {
    if (fp32) {
        const float ch = float(v.c), rh = float(v.r);
        static_cast<HPoint32*>(stage)[i] = HPoint32{ch, rh, float(v.c - double(ch)), float(v.r - double(rh))};
    } else {
        static_cast<HPoint*>(stage)[i] = HPoint{v.c, v.r, 0.0, 0.0};
    }
}

template <int PM>
__device__ __forceinline__ void stage_prep_body(const Model& m, int L, double t, const double* __restrict__ nu,
                                                const YPoint* __restrict__ y, double* __restrict__ mue, void* stage,
                                                int fp32, LogPoint* lstage = nullptr) {
    __shared__ double sh[16];
    double sk = 0.0, se = 0.0;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        const YPoint v = y[i];
        write_stage_point(stage, fp32, i, v);
        if (lstage) lstage[i] = log_point(v.r, 0.0);  // the stage slice carries no derivative
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
template <int PM>
__global__ __launch_bounds__(1024) void k_stage_prep(const Model m, int L, double t, const double* __restrict__ nu,
                                                     const YPoint* __restrict__ y, double* __restrict__ mue,
                                                     void* stage, int fp32, LogPoint* lstage) {
    stage_prep_body<PM>(m, L, t, nu, y, mue, stage, fp32, lstage);
}
template <int PM>
__global__ __launch_bounds__(1024) void k_stage_prep_multi(const PrepDesc* __restrict__ d) {
    const PrepDesc& q = d[blockIdx.x];
    stage_prep_body<PM>(q.m, q.L, q.t, q.nu, q.y, q.mue, q.stage, q.fp32);
}

// ---------------------------------------------------------------- the history integrals
// Bracket search acceleration: per block, bk[q] is the bracket (largest m with
// t_m <= e_q) of the left edge e_q of bucket q of K buckets spaced evenly in
// log2 t over [t_1, t_b].  A target s falls in bucket ~(log2 s - log2 t_1) K /
// span, computed in single precision; the bracket is then found by a binary
// search in double precision between the brackets of neighbouring bucket
// edges, so the result is exact whatever the rounding of the bucket index.
constexpr int kBuckets = 512;

struct Buckets {
    float lt1, inv;  // log2 t_1, K / span
    int on;          // table built (b >= 2)
};

__device__ __forceinline__ int bracket_fast(const double* t, const int* bk, const Buckets& B, int b, double s) {
    if (b <= 1 || s < t[1]) return 0;
    int lo = 0, hi = b;
    if (B.on) {
        int q = int((__log2f(float(s)) - B.lt1) * B.inv);
        q = q < 0 ? 0 : (q > kBuckets ? kBuckets : q);
        lo = bk[q > 0 ? q - 1 : 0];
        hi = bk[q + 2 < kBuckets ? q + 2 : kBuckets] + 1;
        lo = lo > 0 ? lo - 1 : 0;
        hi = hi + 1 < b ? hi + 1 : b;
        while (lo > 0 && t[lo] > s) --lo;    // keep t[lo] <= s <= t[hi]
        while (hi < b && t[hi] < s) ++hi;
    }
    return bracket(t, lo, hi, s);
}

// Pair tiles.  A block owns `rows` consecutive rows j (t' = theta_j t).  Each
// wavefront iteration covers a tile of rows_wave rows x (64 / rows_wave)
// consecutive nodes i; the block's waves split its rows into groups of
// rows_wave and the nodes into `phases` interleaved sets, so one block
// iteration covers all its rows x (cols_wave x phases) nodes.  Tiles of several
// rows keep the 2-D stencil gathers of one instruction within fewer cache lines
// (neighbouring rows read neighbouring history points).  FP64 history: blocks of
// 4 rows (1024 at L = 4096, four per CU in turn), which even out the launch's
// tail better than blocks of 8 (rows below theta = 1/2 cost up to twice the
// others); FP32 history: blocks of 8 rows, whose costs differ less.
template <class HP> struct RowTiles {
    static constexpr int rows = hist_rows_per_block(sizeof(HP) == sizeof(HPoint32) ? 1 : 0);
    static constexpr int rows_wave = rows;
    static constexpr int cols_wave = kWave / rows_wave;
    static constexpr int groups = rows / rows_wave;  // row groups of a block
    static_assert(rows % rows_wave == 0 && kWave % rows_wave == 0, "tile shape");
};


// Tile configuration per history storage type, chosen by measurement at the
// L = 4096 workload: 12 waves per block (3 per SIMD) with the 2-D stencil issued
// first in the iteration, so its reads overlap the stage-slice stencils, for both
// history precisions (with the shared-node tiles below the FP32 kernel fits 3 waves
// per SIMD; before them it ran 8 waves per block, stage-slice stencils first).
template <class HP, int VAR = 0> struct HistCfg {
    // The other theta schemes and the log-R option hold more values per pair:
    // fewer waves per block leave each wave the registers to do so without
    // spilling: 8 waves per block (2 per SIMD) for index Floater-Hormann, 4
    // (1 per SIMD) for the theta schemes and log R, whose 8-wave builds spill
    // and run 1.6-2.8x slower at L = 4096.
    static constexpr int phases = VAR == kVarIndexFH ? 8 : 4;
    static constexpr bool d_first = false;
};
template <> struct HistCfg<HPoint, 0> {
    static constexpr int phases = 12;
    static constexpr bool d_first = true;
};
template <> struct HistCfg<HPoint32, 0> {
    static constexpr int phases = 12;
    static constexpr bool d_first = true;
};
template <class HP, int VAR = 0> constexpr int hist_threads() {
    return RowTiles<HP>::groups * HistCfg<HP, VAR>::phases * kWave;
}

// Per pair (i, j) the kernel forms
//   a = (C,R)(t, theta_i theta_j t)        index Lagrange on the stage slice
//   b = (C,R)(t, phi t)                    phi = theta_j + (1-theta_j) theta_i
//   c = (C,R)(t', theta_i t')              Hermite in t on the row's bracket
//   d = (C,R)(phi t, psi phi t)            psi = theta_j/phi: Lagrange on the two
//                                          bracketing slices, then Hermite in t
// (targets inside the current step use the quadratic through value and d/dt of
// the last slice with a stored derivative and the stage slice), and the nine
// nu-weighted row sums of the forward, transposed and dual equations; one lane
// per row assembles d/dt C(t, theta_j t) = d1C + theta_j d2C and likewise for R.
// LDS of one block: t_n of the stored slices [nb], the bucket table [K+1]
// ints (padded to 8 bytes), when YL the stage slice [L], and when the row
// sums of a row are split over several waves, their partial sums.
__host__ __device__ inline size_t lds_offset_y(int nb) {
    return (size_t(nb > 0 ? nb : 1) * 8 + (kBuckets + 2) * 4 + 15) / 16 * 16;
}
__host__ __device__ inline size_t lds_offset_red(int nb, int L, bool yl) {
    return lds_offset_y(nb) + (yl ? size_t(L) * 16 : 0);
}
// Shared 2-D stencil nodes (default stencil): a wave whose 64 targets bracket the
// same pair of slots and whose stencils lie within kTileNodes consecutive nodes
// reads those nodes of both slots once, one point per lane, into a buffer of its
// own in LDS (2 x kTileNodes points, widened to FP64 for an FP32 history), and its
// stencils then read LDS instead of gathering from global memory.
template <class HP, int VAR> constexpr bool shared_nodes() { return VAR == 0; }
template <class HP, int VAR = 0>
__host__ __device__ inline size_t lds_offset_tile(int nb, int L, bool yl) {
    constexpr int ph = HistCfg<HP, VAR>::phases;
    return lds_offset_red(nb, L, yl) + (ph > 1 ? size_t(RowTiles<HP>::rows) * ph * 9 * 8 : 0);
}
template <class HP, int VAR = 0>
__host__ __device__ inline size_t lds_bytes(int nb, int L, bool yl) {
    constexpr int waves = RowTiles<HP>::groups * HistCfg<HP, VAR>::phases;
    return lds_offset_tile<HP, VAR>(nb, L, yl) +
           (shared_nodes<HP, VAR>() ? size_t(waves) * 2 * kTileNodes * sizeof(HPoint) : 0);
}

template <int S, int PM, class HP, bool YL, int VAR, bool TG = false>
__device__ __forceinline__ void hist_integral_block(const StageArgs& a, int row_block) {
    constexpr bool GEN = VAR != kVarDefault;
    // All arithmetic is FP64, also on an FP32 history: values are widened as
    // they are loaded.  (FP32 arithmetic is no faster than FP64 on this chip
    // without packed instructions, and its rounding, unlike the rounding of the
    // stored values, differs from stage to stage and would reach the embedded
    // error estimate.)
    using HS = hreal_t<HP>;  // storage type of the history
    constexpr int kPhases = HistCfg<HP, VAR>::phases;
    constexpr int kGroups = RowTiles<HP>::groups, kColsPerWave = RowTiles<HP>::cols_wave;
    constexpr int kColStride = kColsPerWave * kPhases;  // nodes one block iteration covers
    extern __shared__ double smem[];
    const int nb = a.nb;
    const int b = nb - 1;
    // TG: more stored slices than LDS holds times for; they are read from global memory
    const int nbl = TG ? 0 : nb;
    double* s_tl = smem;
    int* s_bk = reinterpret_cast<int*>(smem + (nbl > 0 ? nbl : 1));
    if constexpr (!TG)
        for (int q = threadIdx.x; q < nb; q += blockDim.x) s_tl[q] = a.thist[q];
    const double* s_t = TG ? a.thist : s_tl;
    const YPoint* ysrc = a.y;
    if (YL) {
        YPoint* s_y = reinterpret_cast<YPoint*>(reinterpret_cast<char*>(smem) + lds_offset_y(nbl));
        for (int q = threadIdx.x; q < a.L; q += blockDim.x) s_y[q] = a.y[q];
        ysrc = s_y;
    }
    __syncthreads();
    Buckets B{0.0f, 0.0f, 0};
    if (b >= 2) {
        const float lt1 = __log2f(float(s_t[1])), ltb = __log2f(float(s_t[b]));
        const float span = ltb - lt1;
        B.on = span > 0.0f ? 1 : 0;
        B.lt1 = lt1;
        B.inv = B.on ? float(kBuckets) / span : 0.0f;
        if (B.on) {
            for (int q = threadIdx.x; q <= kBuckets; q += blockDim.x) {
                const double e = exp2(double(lt1) + double(q) * double(span) / double(kBuckets));
                int lo = 0;
                if (e >= s_t[b]) lo = b - 1;
                else if (e > 0.0) lo = bracket(s_t, 0, b, e);
                s_bk[q] = lo;
            }
        }
        __syncthreads();
    }

    const int L = a.L;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int grp = wave % kGroups, ph = wave / kGroups;
    const int r = lane / kColsPerWave, cl = lane % kColsPerWave;
    const int row = grp * RowTiles<HP>::rows_wave + r;  // row within the block
    const int jr = row_block * RowTiles<HP>::rows + row;
    if (kPhases == 1 && jr >= L) return;     // whole wave past the end (no later barrier)
    const bool valid = jr < L;
    const int j = valid ? jr : L - 1;
    const HP* hist = static_cast<const HP*>(a.hist);
    const double t = a.t, thj = a.th[j], thcj = a.thc[j], tp = thj * t;
    const double tb = a.tb;

    // Every history value is a weighted sum of two slots: Hermite in t between the
    // bracketing stored slices; inside the current step the quadratic through the
    // last slice with a derivative and the stage slot (weight q2 on both fields of
    // the stage slot, which hold its value, or its FP32 value and remainder); at
    // t = 0 the stage slot alone; with slice 0 as the only stored slice, slice 0.
    const HP* stage = static_cast<const HP*>(a.stage);
    const HP* bslot = nb >= 1 ? hist + size_t(a.slot[b]) * L : stage;
    const HP* slot0 = nb >= 1 ? hist + size_t(a.slot[0]) * L : stage;
    const double hq = t - tb;

    // c family: (C,R)(t', theta_i t') on this row's two slots
    const HP* c0p;
    const HP* c1p;
    double cw0, cw1, cw2, cw3;
    if (nb >= 2 && tp <= tb) {
        const int m = bracket(s_t, 0, b, tp);
        const double h = s_t[m + 1] - s_t[m];
        const double u = (tp - s_t[m]) / h;
        cw0 = 2 * u * u * u - 3 * u * u + 1;
        cw1 = (u * u * u - 2 * u * u + u) * h;
        cw2 = -2 * u * u * u + 3 * u * u;
        cw3 = (u * u * u - u * u) * h;
        c0p = hist + size_t(a.slot[m]) * L;
        c1p = hist + size_t(a.slot[m + 1]) * L;
    } else if (nb >= 1 && tp > tb) {
        const double u = (tp - tb) / hq;
        cw0 = 1.0 - u * u;
        cw1 = hq * (u - u * u);
        cw2 = u * u;
        cw3 = cw2;
        c0p = bslot;
        c1p = stage;
    } else if (nb == 0) {
        cw0 = 1.0, cw1 = 1.0, cw2 = 0.0, cw3 = 0.0;
        c0p = c1p = stage;
    } else {
        cw0 = 1.0, cw1 = 0.0, cw2 = 0.0, cw3 = 0.0;
        c0p = c1p = slot0;
    }
    constexpr bool use_log = var_log(VAR);
    // log mirror rows of the stage slot and of the row's two slots (same offsets as the history)
    // the stage slot may live outside the history (its mirror is a.lstage)
    auto mirror = [&](const HP* slotp) -> const LogPoint* {
        return slotp == stage ? a.lstage : a.lhist + (slotp - hist);
    };
    const LogPoint* lstage = use_log ? a.lstage : nullptr;
    const LogPoint* lc0 = use_log ? mirror(c0p) : nullptr;
    const LogPoint* lc1 = use_log ? mirror(c1p) : nullptr;
    constexpr bool kShared = shared_nodes<HP, VAR>();
    using lds_hp = HPoint __attribute__((address_space(3)));
    // (an address-space cast: the generic pointer to the dynamic LDS becomes an LDS pointer)
    lds_hp* const tile = kShared ? (lds_hp*)(reinterpret_cast<HPoint*>(reinterpret_cast<char*>(smem) +
                                                                   lds_offset_tile<HP, VAR>(nbl, L, YL))) +
                                       wave * 2 * kTileNodes
                                 : nullptr;
    const double* Xa = a.X + size_t(j) * L;          // row j, read forwards
    const double* Xb = a.X + size_t(L - 1 - j) * L;  // row L-1-j, read backwards
    const double* Xdj = a.Xd + size_t(j) * L;

    double S1 = 0, S2 = 0, S3 = 0, S4 = 0, S5 = 0, S6 = 0, S7 = 0, S8 = 0, S9 = 0;
    double c0C = 0.0;
    int mprev = 0;  // FP32 history: this lane's last bracket (its targets s = phi t grow with i)
    const int i0 = cl + kColsPerWave * ph;
    // theta_i and the 2-D coordinate, which start each iteration's dependent chain (the
    // bracket search, then the 2-D stencil), are loaded one iteration ahead (the last
    // iteration reloads node L-1, unused).  Default stencil of up to 10 points only (wider
    // ones have no two registers to spare), and not for an FP32 history with the stage
    // slice in global memory, where it measured about 1% slower.
    constexpr bool kAhead = kShared && S <= 10 && (sizeof(HS) == 8 || YL);
    double th_next = 0.0, xd_next = 0.0;
    if constexpr (kAhead) {
        th_next = a.th[i0 < L ? i0 : L - 1];
        xd_next = Xdj[i0 < L ? i0 : L - 1];
    }
#pragma unroll 1
    for (int i = i0; i < L; i += kColStride) {
        double thi, xd;
        if constexpr (kAhead) {
            thi = th_next;
            xd = xd_next;
            const int inext = i + kColStride < L ? i + kColStride : L - 1;
            th_next = a.th[inext];
            xd_next = Xdj[inext];
        } else {
            thi = a.th[i];
            xd = Xdj[i];
        }
        const double w = a.nu[i], xa = Xa[i], xb = Xb[L - 1 - i];
        double wl[S];
        const double phi = fma(thcj, thi, thj);
        double aC, aR, bC, bR, cC, cR, dC, dR;
        // the stage-slice stencils and the row Hermite
        auto fam_abc = [&]() {
            // a: (t, theta_i theta_j)
            {
                if constexpr (GEN) {
                    const double thci = a.thc[i];
                    const int base = stencil_weights<S, VAR>(a, xa, thi * thj, fma(thi, thcj, thci), wl);
                    interp2<S>(ysrc, base, wl, aC, aR);
                    if constexpr (use_log) aR = log_interp_stage<S>(lstage, base, wl, aR);
                } else {
                    const int base = lagrange<S>(xa, L, wl);
                    if constexpr (kShared) interp2_batched<S>(ysrc, base, wl, aC, aR);
                    else interp2<S>(ysrc, base, wl, aC, aR);
                }
            }
            // b: (t, phi)
            {
                if constexpr (GEN) {
                    const double thci = a.thc[i];
                    const int base = stencil_weights<S, VAR>(a, double(L - 1) - xb, phi, thcj * thci, wl);
                    interp2<S>(ysrc, base, wl, bC, bR);
                    if constexpr (use_log) bR = log_interp_stage<S>(lstage, base, wl, bR);
                } else {
                    const int base = lagrange<S>(double(L - 1) - xb, L, wl);
                    if constexpr (kShared) interp2_batched<S>(ysrc, base, wl, bC, bR);
                    else interp2<S>(ysrc, base, wl, bC, bR);
                }
            }
            // c: (t', theta_i)
            {
                const HP v0 = c0p[i], v1 = c1p[i];
                cC = cw0 * double(v0.c) + cw1 * double(v0.dc) + cw2 * double(v1.c) + cw3 * double(v1.dc);
                cR = cw0 * double(v0.r) + cw1 * double(v0.dr) + cw2 * double(v1.r) + cw3 * double(v1.dr);
                if constexpr (use_log) {
                    // the stage slot's mirror holds a zero derivative: the same four weights apply
                    const LogPoint q0 = lc0[i], q1 = lc1[i];
                    const double l = cw0 * q0.lr + cw1 * q0.lg + cw2 * q1.lr + cw3 * q1.lg;
                    if (!__builtin_isnan(l)) cR = exp(l);
                }
            }
            if (i == 0) c0C = cC;
        };
        // the 2-D stencil on the history
        auto fam_d = [&]() {
            // d: (phi t, psi) on two slots chosen by where s = phi t falls
            {
                double wd[S];
                int base;
                if constexpr (GEN) {
                    double psi = 0.0, psic = 1.0;  // psi = 0/0 := 0 at i = j = 0
                    if (phi > 0.0) {
                        psi = thj / phi;
                        psic = thcj * thi / phi;
                    }
                    base = stencil_weights<S, VAR>(a, xd, psi, psic, wd);
                } else {
                    base = lagrange<S>(xd, L, wd);
                }
                const double s = phi * t;
                const HP* p0;
                const HP* p1;
                double h00, h10, h01, h11;
                int key = -2;  // the slot pair: bracket m, -1 inside the current step, -2 otherwise
                if (nb >= 2 && s <= tb) {
                    int m;
                    if constexpr (sizeof(HS) == 4) {
                        // warm start: the bracket of the lane's previous node, or the one after it
                        m = mprev;
                        if (!(s_t[m] <= s && s < s_t[m + 1])) {
                            if (m + 2 <= b && s_t[m + 1] <= s && s < s_t[m + 2]) m = m + 1;
                            else m = bracket_fast(s_t, s_bk, B, b, s);
                        }
                        mprev = m;
                    } else {
                        m = bracket_fast(s_t, s_bk, B, b, s);
                    }
                    const double h = s_t[m + 1] - s_t[m];
                    const double u = (s - s_t[m]) / h;
                    h00 = 2 * u * u * u - 3 * u * u + 1;
                    h10 = (u * u * u - 2 * u * u + u) * h;
                    h01 = -2 * u * u * u + 3 * u * u;
                    h11 = (u * u * u - u * u) * h;
                    p0 = hist + size_t(a.slot[m]) * L;
                    p1 = hist + size_t(a.slot[m + 1]) * L;
                    key = m;
                } else if (nb >= 1 && s > tb) {
                    const double u = (s - tb) / hq;
                    h00 = 1.0 - u * u;
                    h10 = hq * (u - u * u);
                    h01 = u * u;
                    h11 = h01;
                    p0 = bslot;
                    p1 = stage;
                    key = -1;
                } else if (nb == 0) {
                    h00 = 1.0, h10 = 1.0, h01 = 0.0, h11 = 0.0;
                    p0 = p1 = stage;
                } else {
                    h00 = 1.0, h10 = 0.0, h01 = 0.0, h11 = 0.0;
                    p0 = p1 = slot0;
                }
                double c0, r0, dc0, dr0, c1, r1, dc1, dr1;
                if constexpr (kShared) {
                    // Every lane active (a ragged last tile is not), one slot pair for the whole
                    // wave, and every stencil within kTileNodes nodes of the base of the lane on the
                    // tile's first row and last node, the smallest base of the tile (psi falls with
                    // theta_i and rises with theta_j).
                    __builtin_amdgcn_s_setprio(0);  // the chain is done (raised in the loop below)
                    const int k0 = __builtin_amdgcn_readfirstlane(key);
                    const int bmin = __builtin_amdgcn_readlane(base, kColsPerWave - 1);
                    const int off = base - bmin;
                    const bool ok = key == k0 && off >= 0 && off <= kTileNodes - S;
                    if (__builtin_amdgcn_ballot_w64(true) == ~0ull && __builtin_amdgcn_ballot_w64(!ok) == 0) {
                        // lane q < kTileNodes reads node bmin + q of the first slot, lane
                        // kTileNodes + q the same node of the second; the lanes above 2 kTileNodes idle
                        if (lane < 2 * kTileNodes) {
                            const bool second = lane >= kTileNodes;
                            const int q = second ? lane - kTileNodes : lane;
                            const HP* src = second ? p1 : p0;
                            const HP v = src[bmin + q < L ? bmin + q : L - 1];
                            tile[lane].c = double(v.c);
                            tile[lane].r = double(v.r);
                            tile[lane].dc = double(v.dc);
                            tile[lane].dr = double(v.dr);
                        }
                        // LDS operations of one wave take effect in program order: the fences
                        // only keep the compiler from moving the reads above the writes
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                        shared_stencil<S>(tile, off, wd, c0, r0, dc0, dr0, c1, r1, dc1, dr1);
                    } else {
                        gathered_stencil<S>(p0, p1, base, wd, c0, r0, dc0, dr0, c1, r1, dc1, dr1);
                    }
                } else {
                    interp4<S>(p0, base, wd, c0, r0, dc0, dr0);
                    // FP32 storage: values are widened as they arrive, so the second slot's
                    // gathers wait for the first (keeps the widened values within registers)
                    if constexpr (sizeof(HS) == 4) __builtin_amdgcn_sched_barrier(0);
                    interp4<S>(p1, base, wd, c1, r1, dc1, dr1);
                }
                dC = h00 * c0 + h10 * dc0 + h01 * c1 + h11 * dc1;
                dR = h00 * r0 + h10 * dr0 + h01 * r1 + h11 * dr1;
                if constexpr (use_log) {
                    double lv0, ld0, lv1, ld1;
                    log_interp_slot<S>(mirror(p0), base, wd, lv0, ld0);
                    log_interp_slot<S>(mirror(p1), base, wd, lv1, ld1);
                    const double l = h00 * lv0 + h10 * ld0 + h01 * lv1 + h11 * ld1;
                    if (!__builtin_isnan(l)) dR = exp(l);
                }
            }
        };
        if constexpr (HistCfg<HP, VAR>::d_first) {
            // the wave issues ahead of the block's other waves on its SIMD until its 2-D
            // stencil's addresses are known: the bracket search and the slot indices are a
            // chain of dependent reads, and its loads then go out sooner
            if constexpr (kShared) __builtin_amdgcn_s_setprio(2);
            fam_d();
            fam_abc();
        } else {
            fam_abc();
            fam_d();
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
    double Sv[9] = {S1, S2, S3, S4, S5, S6, S7, S8, S9};
#pragma unroll
    for (int k = 0; k < 9; ++k) {  // sum over the lanes of the row (fixed order)
#pragma unroll
        for (int off = kColsPerWave / 2; off > 0; off >>= 1) Sv[k] += __shfl_xor(Sv[k], off, kWave);
    }
    bool assemble = cl == 0;
    if (kPhases > 1) {  // rows split over waves: partial sums through LDS, summed in phase order
        double* red = reinterpret_cast<double*>(reinterpret_cast<char*>(smem) + lds_offset_red(nbl, L, YL));
        __syncthreads();  // every wave is done with the stage slice region and the bracket tables
        if (cl == 0) {
#pragma unroll
            for (int k = 0; k < 9; ++k) red[(row * kPhases + ph) * 9 + k] = Sv[k];
        }
        __syncthreads();
        assemble = cl == 0 && ph == 0;
        if (assemble) {
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                double v = red[(row * kPhases) * 9 + k];
                for (int q = 1; q < kPhases; ++q) v += red[(row * kPhases + q) * 9 + k];
                Sv[k] = v;
            }
        }
    }
    if (assemble && valid) {
        const double mu = a.mue[0];
        const YPoint y0 = a.y[0], yj = a.y[j];
        const double T = a.m.T, be = a.m.beta0;
        const double d1C = -mu * yj.c + t * (thj * Sv[0] + thj * Sv[1] + thcj * Sv[2]) + be * fD1<PM>(a.m, y0.c) * c0C;
        const double d1R = -mu * yj.r + t * thcj * Sv[3];
        const double mup = T + t * thj * Sv[8] + be * fD1<PM>(a.m, c0C) * c0C;
        const double d2C = -mup * yj.c + t * (thj * Sv[4] + thj * Sv[5] + thcj * Sv[6]) + 2.0 * T * yj.r +
                           be * fD1<PM>(a.m, c0C) * y0.c;
        const double d2R = mup * yj.r - t * thcj * Sv[7];
        double oc = d1C + thj * d2C, orr = d1R + thj * d2R;
        if (j == L - 1) {
            a.diag[0] = oc;
            a.diag[1] = orr;
            oc = 0.0;
            orr = 0.0;
        }
        a.kout[j] = YPoint{oc, orr};
        if (a.store) {
            HP* st = static_cast<HP*>(a.store);
            st[j].dc = HS(oc);
            st[j].dr = HS(orr);
            // the log mirror of the slot from its stored values (a slice not yet appended
            // gets it again when it is)
            if constexpr (use_log) a.lhist[(st - hist) + j] = log_point(double(st[j].r), double(HS(orr)));
        }
    }
}

// One instance: the stage arguments travel by value.
template <int S, int PM, class HP, bool YL, int VAR, bool TG = false>
__global__ __launch_bounds__((hist_threads<HP, VAR>())) void k_hist_integral(const StageArgs a) {
    hist_integral_block<S, PM, HP, YL, VAR, TG>(a, blockIdx.x);
}

// Many instances in one launch (serving): block b belongs to the instance q
// with first_block[q] <= b < first_block[q+1]; instances may differ in L, M,
// t and history.  The dynamic LDS is sized for the largest nb of the batch.
template <int S, int PM, class HP, bool YL>
__global__ __launch_bounds__(hist_threads<HP>()) void k_hist_integral_multi(const StageArgs* __restrict__ args,
                                                                            const int* __restrict__ first_block,
                                                                            int n_inst) {
    int lo = 0, hi = n_inst;  // first_block[lo] <= b < first_block[hi]
    const int b = blockIdx.x;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first_block[mid] <= b) lo = mid;
        else hi = mid;
    }
    hist_integral_block<S, PM, HP, YL, kVarDefault>(args[lo], b - first_block[lo]);
}

// ---------------------------------------------------------------- RK stage combinations
struct Coef10 {
    double v[10];
};

// ys = y0 + dt sum_{l < nk} a_l k_l; the diagonal point is pinned to (1, 1).
__device__ __forceinline__ void rk_combine_point(int i, int L, const YPoint* __restrict__ y0,
                                                 const YPoint* __restrict__ k, int nk, const double* a, double dt,
                                                 YPoint* __restrict__ ys) {
    if (i >= L) return;
    YPoint acc = y0[i];
    for (int l = 0; l < nk; ++l) {
        const double f = dt * a[l];
        const YPoint kv = k[size_t(l) * L + i];
        acc.c = fma(f, kv.c, acc.c);
        acc.r = fma(f, kv.r, acc.r);
    }
    if (i == L - 1) acc = YPoint{1.0, 1.0};
    ys[i] = acc;
}
__global__ void k_rk_combine(int L, const YPoint* __restrict__ y0, const YPoint* __restrict__ k, int nk,
                             const Coef10 a, double dt, YPoint* __restrict__ ys) {
    rk_combine_point(blockIdx.x * blockDim.x + threadIdx.x, L, y0, k, nk, a.v, dt, ys);
}
__global__ __launch_bounds__(kCombineBlock) void k_rk_combine_multi(const CombineDesc* __restrict__ d,
                                                                    const int* __restrict__ first_block, int n) {
    int lo = 0, hi = n;
    const int b = blockIdx.x;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first_block[mid] <= b) lo = mid;
        else hi = mid;
    }
    const CombineDesc& q = d[lo];
    rk_combine_point((b - first_block[lo]) * blockDim.x + threadIdx.x, q.L, q.y0, q.k, q.nk, q.a, q.dt, q.ys);
}

// ynew = y0 + dt sum b_l k_l and eps = sum_i |dt sum e_l k_l| over both fields
// (Sec. 3.5), one block so that the sum has a fixed order.
__device__ __forceinline__ void rk_finish_body(int L, const YPoint* __restrict__ y0, const YPoint* __restrict__ k,
                                               int nk, const double* bw, const double* ew, double dt,
                                               YPoint* __restrict__ ynew, double* __restrict__ eps_out) {
    __shared__ double sh[16];
    double sum = 0.0;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        YPoint acc = y0[i];
        double ec = 0.0, er = 0.0;
        for (int l = 0; l < nk; ++l) {
            const YPoint kv = k[size_t(l) * L + i];
            const double f = dt * bw[l];
            acc.c = fma(f, kv.c, acc.c);
            acc.r = fma(f, kv.r, acc.r);
            ec = fma(ew[l], kv.c, ec);
            er = fma(ew[l], kv.r, er);
        }
        if (i == L - 1) acc = YPoint{1.0, 1.0};
        ynew[i] = acc;
        sum += fabs(dt * ec) + fabs(dt * er);
    }
    sum = block_sum(sum, sh);
    if (threadIdx.x == 0) eps_out[0] = sum;
}
__global__ __launch_bounds__(1024) void k_rk_finish(int L, const YPoint* __restrict__ y0,
                                                    const YPoint* __restrict__ k, int nk, const Coef10 bw,
                                                    const Coef10 ew, double dt, YPoint* __restrict__ ynew,
                                                    double* __restrict__ eps_out) {
    rk_finish_body(L, y0, k, nk, bw.v, ew.v, dt, ynew, eps_out);
}
__global__ __launch_bounds__(1024) void k_rk_finish_multi(const FinishDesc* __restrict__ d) {
    const FinishDesc& q = d[blockIdx.x];
    rk_finish_body(q.L, q.y0, q.k, q.nk, q.b, q.e, q.dt, q.ynew, q.eps);
}

// Accepting a step (Sec. 3.2): the new state goes into its slice slot as (C, R) (the
// derivative half is written by a first-same-as-last scheme's last stage, else by
// the next step's first stage) and becomes the state; with a first-same-as-last
// scheme the last stage's derivative becomes the next step's first; thread 0 writes
// the slice's time and slot to the device copies of the ordered history.
template <class HP>
__global__ void k_accept(const AcceptArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        a.thist[a.M] = a.t_new;
        a.slots[a.M] = a.slot_new;
    }
    if (i >= a.L) return;
    HP* dst = static_cast<HP*>(a.slot_dst);
    const YPoint v = a.ynew[i];
    const hreal_t<HP> r = hreal_t<HP>(v.r);
    dst[i].c = hreal_t<HP>(v.c);
    dst[i].r = r;
    a.y0[i] = v;
    if (a.k_first) a.k_first[i] = a.k_last[i];
    // log mirror from the stored values; dr is the derivative a first-same-as-last
    // stage stored already, else a placeholder the next first stage overwrites
    if (a.lslot) a.lslot[i] = log_point(double(r), double(dst[i].dr));
}

template <class HP>
__global__ void k_log_mirror(int L, int count, const int* __restrict__ slot, const HP* __restrict__ hist,
                             LogPoint* __restrict__ lhist) {
    const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= size_t(count) * L) return;
    const size_t off = size_t(slot[idx / L]) * L + idx % L;
    lhist[off] = log_point(double(hist[off].r), double(hist[off].dr));
}

template <class HP>
__global__ void k_load_state(int L, const HP* __restrict__ src, YPoint* __restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L) return;
    y[i] = YPoint{double(src[i].c), double(src[i].r)};
}

// ---------------------------------------------------------------- sparsification residual
__device__ __forceinline__ HPoint up(const HPoint& v) { return v; }
__device__ __forceinline__ HPoint up(const HPoint32& v) {
    return HPoint{double(v.c), double(v.r), double(v.dc), double(v.dr)};
}
// eps_n = sum_i |Delta^C_n(theta_i)| + |Delta^R_n(theta_i)| with Delta the Hermite
// integral over [t_{n-1}, t_{n+1}] with slice n minus the one without (Sec. 3.6).
__device__ __forceinline__ double herm_int(double h, double ya, double da, double yb, double db) {
    return h * (ya + yb) * 0.5 + h * h * (da - db) * (1.0 / 12.0);
}
// Rounding allowance of an FP32 history: a stored value differs from the FP64
// value it was rounded from by at most u |stored| (u = 2^-24), so the residual
// of the stored values differs from the residual of the FP64 values by at most
// the sum over points of u times |coefficient| |stored| over the six values of
// each field.  The coefficients of the residual in the values at n-1, n, n+1
// are -h2/2, h3/2, -h1/2 and in the derivatives (h1^2-h3^2)/12,
// (h2^2-h1^2)/12, (h3^2-h2^2)/12.
template <class HP> struct RoundingAllowance {
    static constexpr bool on = false;
};
template <> struct RoundingAllowance<HPoint32> {
    static constexpr bool on = true;
};
constexpr double kUnitRoundoff32 = 5.9604644775390625e-8;  // 2^-24

// eps_n = sum_i |Delta^C_i| + |Delta^R_i| for candidate n (Sec. 3.6), with
// Delta = H[n-1,n] + H[n,n+1] - H[n-1,n+1].  For an FP32 history the rounding
// allowance is subtracted (never below zero), so a slice is kept only if its
// residual exceeds what the storage precision can resolve by eps/10.
//
// A block owns a run of kSpK consecutive candidates and a chunk of kSpChunk
// nodes: each thread slides a three-slice window along the run at its nodes,
// so every slice of the run is read once (plus the two slices around it)
// instead of once per candidate that touches it.  The partial sums of the
// chunks go to part[chunk][n] (and the rounding allowance to bnd[chunk][n]);
// k_sparsify_final adds the chunks in a fixed order.
constexpr int kSpK = 16;        // candidates per block
constexpr int kSpNpt = 4;       // nodes per thread
constexpr int kSpThreads = 256;
constexpr int kSpChunk = kSpThreads * kSpNpt;

template <class HP>
__global__ __launch_bounds__(kSpThreads) void k_sparsify_part(int L, int first, int count, int stride,
                                                              const double* __restrict__ thist,
                                                              const int* __restrict__ slot,
                                                              const HP* __restrict__ hist, double* __restrict__ part,
                                                              double* __restrict__ bnd) {
    __shared__ double red[kSpThreads / kWave][kSpK][2];
    constexpr bool fp32 = RoundingAllowance<HP>::on;
    const int n0 = first + int(blockIdx.x) * kSpK;       // first candidate of the run
    const int kc = min(kSpK, first + count - n0);        // candidates in this run
    const int i0 = int(blockIdx.y) * kSpChunk + int(threadIdx.x);
    double e[kSpK], b[kSpK];
#pragma unroll
    for (int c = 0; c < kSpK; ++c) e[c] = b[c] = 0.0;
    // the run's slices n0-1 .. n0+kc (uniform per block)
    HPoint va[kSpNpt], vc[kSpNpt];
    const HP* s0 = hist + size_t(slot[n0 - 1]) * L;
    const HP* s1 = hist + size_t(slot[n0]) * L;
#pragma unroll
    for (int q = 0; q < kSpNpt; ++q) {
        const int i = i0 + q * kSpThreads;
        va[q] = vc[q] = HPoint{0.0, 0.0, 0.0, 0.0};
        if (i < L) {
            va[q] = up(s0[i]);
            vc[q] = up(s1[i]);
        }
    }
#pragma unroll
    for (int c = 0; c < kSpK; ++c) {
        if (c < kc) {
            const int n = n0 + c;
            const double tm = thist[n - 1], tn = thist[n], tp = thist[n + 1];
            const double h1 = tn - tm, h2 = tp - tn, h3 = tp - tm;
            const HP* sb = hist + size_t(slot[n + 1]) * L;
            const double ka = 0.5 * h2, kcn = 0.5 * h3, kb = 0.5 * h1;
            const double qa = fabs(h1 * h1 - h3 * h3) * (1.0 / 12.0), qc = fabs(h2 * h2 - h1 * h1) * (1.0 / 12.0),
                         qb = fabs(h3 * h3 - h2 * h2) * (1.0 / 12.0);
#pragma unroll
            for (int q = 0; q < kSpNpt; ++q) {
                const int i = i0 + q * kSpThreads;
                HPoint vb = HPoint{0.0, 0.0, 0.0, 0.0};
                if (i < L) vb = up(sb[i]);
                const HPoint& A = va[q];
                const HPoint& Cc = vc[q];
                const double dc = herm_int(h1, A.c, A.dc, Cc.c, Cc.dc) + herm_int(h2, Cc.c, Cc.dc, vb.c, vb.dc) -
                                  herm_int(h3, A.c, A.dc, vb.c, vb.dc);
                const double dr = herm_int(h1, A.r, A.dr, Cc.r, Cc.dr) + herm_int(h2, Cc.r, Cc.dr, vb.r, vb.dr) -
                                  herm_int(h3, A.r, A.dr, vb.r, vb.dr);
                e[c] += fabs(dc) + fabs(dr);
                if (fp32)
                    b[c] += ka * (fabs(A.c) + fabs(A.r)) + kcn * (fabs(Cc.c) + fabs(Cc.r)) +
                            kb * (fabs(vb.c) + fabs(vb.r)) + qa * (fabs(A.dc) + fabs(A.dr)) +
                            qc * (fabs(Cc.dc) + fabs(Cc.dr)) + qb * (fabs(vb.dc) + fabs(vb.dr));
                va[q] = vc[q];
                vc[q] = vb;
            }
        }
    }
    // block sums of the run's candidates, in a fixed order
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int c = 0; c < kSpK; ++c) {
        const double se = wave_sum(e[c]);
        const double sb = fp32 ? wave_sum(b[c]) : 0.0;
        if (lane == 0) {
            red[w][c][0] = se;
            red[w][c][1] = sb;
        }
    }
    __syncthreads();
    if (int(threadIdx.x) < kc) {
        const int c = threadIdx.x;
        double se = 0.0, sb = 0.0;
        for (int q = 0; q < kSpThreads / kWave; ++q) {
            se += red[q][c][0];
            sb += red[q][c][1];
        }
        part[size_t(blockIdx.y) * stride + n0 + c] = se;
        if (fp32) bnd[size_t(blockIdx.y) * stride + n0 + c] = sb;
    }
}

// eps_n from the chunks' partial sums, in chunk order.
__global__ void k_sparsify_final(int first, int count, int chunks, int stride, int fp32,
                                 const double* __restrict__ part, const double* __restrict__ bnd,
                                 double* __restrict__ eps_n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int n = first + k;
    double e = 0.0, bd = 0.0;
    for (int q = 0; q < chunks; ++q) {
        e += part[size_t(q) * stride + n];
        if (fp32) bd += bnd[size_t(q) * stride + n];
    }
    if (fp32) {
        bd *= kUnitRoundoff32;
        e = e > bd ? e - bd : 0.0;
    }
    eps_n[n] = e;
}

// ---------------------------------------------------------------- observables and copies
template <int PM, class HP>
__global__ __launch_bounds__(256) void k_slice_observables(const Model m, int L, const double* __restrict__ nu,
                                                           const double* __restrict__ thist,
                                                           const int* __restrict__ slot, const HP* __restrict__ hist,
                                                           double* __restrict__ E, double* __restrict__ mu) {
    __shared__ double sh[16];
    const int n = blockIdx.x;
    const HP* p = hist + size_t(slot[n]) * L;
    double sk = 0.0, se = 0.0;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        const HPoint v = up(p[i]);
        const double d1 = fD1<PM>(m, v.c), d2 = fD2<PM>(m, v.c);
        sk = fma(nu[i], d2 * v.r * v.c + d1 * v.r, sk);
        se = fma(nu[i], d1 * v.r, se);
    }
    sk = block_sum(sk, sh);
    se = block_sum(se, sh);
    if (threadIdx.x == 0) {
        const double t = thist[n];
        const double c0 = double(p[0].c);
        if (mu) mu[n] = m.T + t * sk + m.beta0 * fD1<PM>(m, c0) * c0;
        if (E) E[n] = -t * se - m.beta0 * fF<PM>(m, c0);
    }
}

template <class HP>
__global__ void k_pack(int L, int count, int field, const int* __restrict__ slot, const HP* __restrict__ hist,
                       double* __restrict__ dst) {
    const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= size_t(count) * L) return;
    const int n = int(idx / L), i = int(idx % L);
    const HPoint v = up(hist[size_t(slot[n]) * L + i]);
    dst[idx] = field == 0 ? v.c : field == 1 ? v.r : field == 2 ? v.dc : v.dr;
}

template <class HP>
__global__ void k_unpack(int L, int count, const double* __restrict__ C, const double* __restrict__ R,
                         const double* __restrict__ dC, const double* __restrict__ dR,
                         const int* __restrict__ slot, HP* __restrict__ hist) {
    const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= size_t(count) * L) return;
    const int n = int(idx / L), i = int(idx % L);
    using R_ = hreal_t<HP>;
    hist[size_t(slot[n]) * L + i] = HP{R_(C[idx]), R_(R[idx]), R_(dC[idx]), R_(dR[idx])};
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
hipError_t launch_coords(const GridArgs& g, hipStream_t st) {
    hipLaunchKernelGGL(k_coords, dim3(nblk(g.L, 256), g.L), dim3(256), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_stage_prep(const Model& m, int L, double t, const double* nu, const YPoint* y, double* mue,
                             void* stage, int fp32, LogPoint* lstage, hipStream_t st) {
    if (m.pmax <= 4)
        hipLaunchKernelGGL(k_stage_prep<4>, dim3(1), dim3(1024), 0, st, m, L, t, nu, y, mue, stage, fp32, lstage);
    else
        hipLaunchKernelGGL(k_stage_prep<DMFE_MAX_P>, dim3(1), dim3(1024), 0, st, m, L, t, nu, y, mue, stage, fp32,
                           lstage);
    return hipGetLastError();
}

// Largest dynamic LDS a block may use on this device (queried once).
static size_t max_lds() {
    static size_t v = 0;
    if (v == 0) {
        int dev = 0, b = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&b, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && b > 0)
            v = size_t(b);
        else
            v = 65536;
    }
    return v;
}

// Raise a kernel's dynamic-LDS limit when a launch needs more than the default
// 64 KB.  The attribute is set once per (device, kernel) for the largest size
// seen so far, not on every launch.
template <class K>
static void allow_lds(K kernel, size_t bytes) {
    if (bytes <= 65536) return;
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, size_t> done;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const auto key = std::make_pair(dev, reinterpret_cast<const void*>(kernel));
    std::lock_guard<std::mutex> lk(mu);
    auto it = done.find(key);
    if (it != done.end() && it->second >= bytes) return;
    if (hipFuncSetAttribute(key.second, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)) == hipSuccess)
        done[key] = bytes;
}

template <int S, class HP, bool YL, int VAR, bool TG = false>
static void launch_gen(const StageArgs& a, dim3 grid, hipStream_t st) {
    const size_t lds = lds_bytes<HP, VAR>(TG ? 0 : a.nb, a.L, YL);
    allow_lds(k_hist_integral<S, DMFE_MAX_P, HP, YL, VAR, TG>, lds);
    hipLaunchKernelGGL((k_hist_integral<S, DMFE_MAX_P, HP, YL, VAR, TG>), grid, dim3(hist_threads<HP, VAR>()), lds,
                       st, a);
}
// the option schemes (theta stencils, Floater-Hormann, log-R), one instantiation each
template <int S, class HP, bool YL, bool TG>
static void launch_gen_var(const StageArgs& a, dim3 grid, hipStream_t st) {
    const bool fh = a.interp == DMFE_INTERP_INDEX_FH;
    const bool th = a.interp == DMFE_INTERP_THETA_LAGRANGE || a.interp == DMFE_INTERP_THETA_FH;
    if (!a.log_r) {
        if (fh) launch_gen<S, HP, YL, kVarIndexFH, TG>(a, grid, st);
        else launch_gen<S, HP, YL, kVarTheta, TG>(a, grid, st);
    } else if (fh) {
        launch_gen<S, HP, YL, kVarIndexFHLog, TG>(a, grid, st);
    } else if (th) {
        launch_gen<S, HP, YL, kVarThetaLog, TG>(a, grid, st);
    } else {
        launch_gen<S, HP, YL, kVarIndexLagrangeLog, TG>(a, grid, st);
    }
}
template <int S, class HP, bool YL>
static void launch_hi_shy(const StageArgs& a, size_t lds, hipStream_t st) {
    const dim3 grid(nblk(a.L, RowTiles<HP>::rows)), block(hist_threads<HP>());
    if (a.interp != DMFE_INTERP_INDEX_LAGRANGE || a.log_r) {
        launch_gen_var<S, HP, YL, false>(a, grid, st);
    } else if (a.m.pmax <= 4) {
        allow_lds(k_hist_integral<S, 4, HP, YL, kVarDefault>, lds);
        hipLaunchKernelGGL((k_hist_integral<S, 4, HP, YL, kVarDefault>), grid, block, lds, st, a);
    } else {
        allow_lds(k_hist_integral<S, DMFE_MAX_P, HP, YL, kVarDefault>, lds);
        hipLaunchKernelGGL((k_hist_integral<S, DMFE_MAX_P, HP, YL, kVarDefault>), grid, block, lds, st, a);
    }
}
template <int S, class HP>
static hipError_t launch_hi_sh(const StageArgs& a, hipStream_t st) {
    const size_t with_y = lds_bytes<HP>(a.nb, a.L, true);
    const size_t without_y = lds_bytes<HP>(a.nb, a.L, false);
    if (with_y <= max_lds()) {
        launch_hi_shy<S, HP, true>(a, with_y, st);
    } else if (without_y <= max_lds()) {
        launch_hi_shy<S, HP, false>(a, without_y, st);
    } else {
        // more stored slices than LDS holds times for (with 160 KB of LDS, about 17K with the default
        // stencil, 20K with the others): they are read from global memory
        const size_t lds = lds_bytes<HP>(0, a.L, false);
        const dim3 grid(nblk(a.L, RowTiles<HP>::rows)), block(hist_threads<HP>());
        if (a.interp != DMFE_INTERP_INDEX_LAGRANGE || a.log_r) {
            launch_gen_var<S, HP, false, true>(a, grid, st);
        } else if (a.m.pmax <= 4) {
            allow_lds(k_hist_integral<S, 4, HP, false, kVarDefault, true>, lds);
            hipLaunchKernelGGL((k_hist_integral<S, 4, HP, false, kVarDefault, true>), grid, block, lds, st, a);
        } else {
            allow_lds(k_hist_integral<S, DMFE_MAX_P, HP, false, kVarDefault, true>, lds);
            hipLaunchKernelGGL((k_hist_integral<S, DMFE_MAX_P, HP, false, kVarDefault, true>), grid, block, lds, st,
                               a);
        }
    }
    return hipGetLastError();
}
template <int S>
static hipError_t launch_hi_s(const StageArgs& a, hipStream_t st) {
    return a.fp32 ? launch_hi_sh<S, HPoint32>(a, st) : launch_hi_sh<S, HPoint>(a, st);
}

hipError_t launch_hist_integral(const StageArgs& a, int s, hipStream_t st) {
    switch (s) {
    case 4: return launch_hi_s<4>(a, st);
    case 6: return launch_hi_s<6>(a, st);
    case 8: return launch_hi_s<8>(a, st);
    case 10: return launch_hi_s<10>(a, st);
    case 12: return launch_hi_s<12>(a, st);
    case 14: return launch_hi_s<14>(a, st);
    case 16: return launch_hi_s<16>(a, st);
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

hipError_t launch_accept(const AcceptArgs& a, int fp32, hipStream_t st) {
    if (fp32)
        hipLaunchKernelGGL(k_accept<HPoint32>, dim3(nblk(a.L, 256)), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_accept<HPoint>, dim3(nblk(a.L, 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_log_mirror(int L, int count, const int* slot, const void* hist, int fp32, LogPoint* lhist,
                             hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const dim3 g(nblk(size_t(count) * L, 256));
    if (fp32)
        hipLaunchKernelGGL(k_log_mirror<HPoint32>, g, dim3(256), 0, st, L, count, slot,
                           static_cast<const HPoint32*>(hist), lhist);
    else
        hipLaunchKernelGGL(k_log_mirror<HPoint>, g, dim3(256), 0, st, L, count, slot, static_cast<const HPoint*>(hist),
                           lhist);
    return hipGetLastError();
}

hipError_t launch_load_state(int L, const void* slot_src, int fp32, YPoint* y, hipStream_t st) {
    if (fp32)
        hipLaunchKernelGGL(k_load_state<HPoint32>, dim3(nblk(L, 256)), dim3(256), 0, st, L,
                           static_cast<const HPoint32*>(slot_src), y);
    else
        hipLaunchKernelGGL(k_load_state<HPoint>, dim3(nblk(L, 256)), dim3(256), 0, st, L,
                           static_cast<const HPoint*>(slot_src), y);
    return hipGetLastError();
}

int sparsify_chunks(int L) { return (L + kSpChunk - 1) / kSpChunk; }

hipError_t launch_sparsify_residual(int L, int first, int count, const double* thist, const int* slot,
                                    const void* hist, int fp32, double* eps_n, double* part, int stride,
                                    hipStream_t st) {
    if (count <= 0) return hipSuccess;
    if (first < 1 || first + count + 1 > stride) return hipErrorInvalidValue;  // slices first-1 .. first+count
    const int chunks = sparsify_chunks(L);
    const dim3 grid(unsigned((count + kSpK - 1) / kSpK), unsigned(chunks));
    double* bnd = part + size_t(chunks) * stride;
    if (fp32)
        hipLaunchKernelGGL(k_sparsify_part<HPoint32>, grid, dim3(kSpThreads), 0, st, L, first, count, stride, thist,
                           slot, static_cast<const HPoint32*>(hist), part, bnd);
    else
        hipLaunchKernelGGL(k_sparsify_part<HPoint>, grid, dim3(kSpThreads), 0, st, L, first, count, stride, thist,
                           slot, static_cast<const HPoint*>(hist), part, bnd);
    hipLaunchKernelGGL(k_sparsify_final, dim3(nblk(count, 256)), dim3(256), 0, st, first, count, chunks, stride, fp32,
                       part, bnd, eps_n);
    return hipGetLastError();
}

template <class HP>
static void obs_launch(const Model& m, int L, const double* nu, int count, const double* thist, const int* slot,
                       const HP* hist, double* E, double* mu, hipStream_t st) {
    if (m.pmax <= 4)
        hipLaunchKernelGGL((k_slice_observables<4, HP>), dim3(count), dim3(256), 0, st, m, L, nu, thist, slot, hist, E,
                           mu);
    else
        hipLaunchKernelGGL((k_slice_observables<DMFE_MAX_P, HP>), dim3(count), dim3(256), 0, st, m, L, nu, thist, slot,
                           hist, E, mu);
}

hipError_t launch_slice_observables(const Model& m, int L, const double* nu, int count, const double* thist,
                                    const int* slot, const void* hist, int fp32, double* E, double* mu,
                                    hipStream_t st) {
    if (count <= 0) return hipSuccess;
    if (fp32) obs_launch(m, L, nu, count, thist, slot, static_cast<const HPoint32*>(hist), E, mu, st);
    else obs_launch(m, L, nu, count, thist, slot, static_cast<const HPoint*>(hist), E, mu, st);
    return hipGetLastError();
}

hipError_t launch_pack_history(int L, int count, int field, const int* slot, const void* hist, int fp32,
                               double* dst, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const dim3 g(nblk(size_t(count) * L, 256));
    if (fp32)
        hipLaunchKernelGGL(k_pack<HPoint32>, g, dim3(256), 0, st, L, count, field, slot,
                           static_cast<const HPoint32*>(hist), dst);
    else
        hipLaunchKernelGGL(k_pack<HPoint>, g, dim3(256), 0, st, L, count, field, slot, static_cast<const HPoint*>(hist),
                           dst);
    return hipGetLastError();
}

hipError_t launch_unpack_history(int L, int count, const double* C, const double* R, const double* dC,
                                 const double* dR, const int* slot, void* hist, int fp32, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const dim3 g(nblk(size_t(count) * L, 256));
    if (fp32)
        hipLaunchKernelGGL(k_unpack<HPoint32>, g, dim3(256), 0, st, L, count, C, R, dC, dR, slot,
                           static_cast<HPoint32*>(hist));
    else
        hipLaunchKernelGGL(k_unpack<HPoint>, g, dim3(256), 0, st, L, count, C, R, dC, dR, slot,
                           static_cast<HPoint*>(hist));
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

hipError_t launch_rk_combine_multi(const CombineDesc* d, const int* first_block, int n, int total_blocks,
                                   hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rk_combine_multi, dim3(total_blocks), dim3(kCombineBlock), 0, st, d, first_block, n);
    return hipGetLastError();
}

hipError_t launch_stage_prep_multi(const PrepDesc* d, int n, int pmax, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (pmax <= 4) hipLaunchKernelGGL(k_stage_prep_multi<4>, dim3(n), dim3(1024), 0, st, d);
    else hipLaunchKernelGGL(k_stage_prep_multi<DMFE_MAX_P>, dim3(n), dim3(1024), 0, st, d);
    return hipGetLastError();
}

template <int S, class HP>
static void hist_multi_launch(const StageArgs* d, const int* fb, int n, int blocks, int pmax, size_t lds,
                              hipStream_t st) {
    allow_lds(k_hist_integral_multi<S, 4, HP, false>, lds);
    allow_lds(k_hist_integral_multi<S, DMFE_MAX_P, HP, false>, lds);
    if (pmax <= 4)
        hipLaunchKernelGGL((k_hist_integral_multi<S, 4, HP, false>), dim3(blocks), dim3(hist_threads<HP>()), lds,
                           st, d, fb, n);
    else
        hipLaunchKernelGGL((k_hist_integral_multi<S, DMFE_MAX_P, HP, false>), dim3(blocks),
                           dim3(hist_threads<HP>()), lds, st, d, fb, n);
}

hipError_t launch_hist_integral_multi(const StageArgs* d, const int* first_block, int n, int total_blocks, int s,
                                      int pmax, int fp32, int nb_max, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (s != 10) return hipErrorInvalidValue;  // the pool serves the default stencil
    if (fp32)
        hist_multi_launch<10, HPoint32>(d, first_block, n, total_blocks, pmax, lds_bytes<HPoint32>(nb_max, 0, false), st);
    else
        hist_multi_launch<10, HPoint>(d, first_block, n, total_blocks, pmax, lds_bytes<HPoint>(nb_max, 0, false), st);
    return hipGetLastError();
}

hipError_t launch_rk_finish_multi(const FinishDesc* d, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rk_finish_multi, dim3(n), dim3(1024), 0, st, d);
    return hipGetLastError();
}

}  // namespace dmfe
