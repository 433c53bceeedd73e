// Host core of libdmfe: the C-ABI declared in include/dmfe.h.
//
// The host owns only scalar control (the step-size controller of Sec. 3.5,
// the greedy selection of Sec. 3.6, bookkeeping of the slice order); every
// array operation of the solver runs in the kernels of kernels_theta.hip and
// kernels_uniform.hip on the handle's stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "handle.h"

namespace dmfe {
namespace core {

namespace {
thread_local std::string g_last_error;
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error() { return g_last_error.c_str(); }

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Dormand-Prince 5(4) (Sec. 3.5).
Tableau make_dp5() {
    Tableau T;
    T.S = 7;
    const double A[7][7] = {
        {0, 0, 0, 0, 0, 0, 0},
        {1.0 / 5, 0, 0, 0, 0, 0, 0},
        {3.0 / 40, 9.0 / 40, 0, 0, 0, 0, 0},
        {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0, 0},
        {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0, 0},
        {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0, 0},
        {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0}};
    const double bhat[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640, -92097.0 / 339200, 187.0 / 2100,
                            1.0 / 40};
    const double c[7] = {0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1, 1};
    for (int i = 0; i < 7; ++i) {
        for (int j = 0; j < 7; ++j) T.A[i][j] = A[i][j];
        T.b[i] = A[6][i];
        T.e[i] = A[6][i] - bhat[i];
        T.c[i] = c[i];
    }
    T.fsal = true;
    return T;
}

// SSPRK(10,4) (Sec. 3.5) in Butcher form: five Euler stages of dt/6, the
// combination 3/5 u + 2/5 q, four more Euler stages, weights 1/10.  The
// embedded third-order weights minimise |bhat|_2 over stages 1..9 subject to
// the four third-order conditions (sum bhat = 1, bhat.c = 1/2, bhat.c^2 = 1/3,
// bhat.Ac = 1/6): bhat = M^T (M M^T)^{-1} r.
Tableau make_ssprk104() {
    Tableau T;
    T.S = 10;
    for (int k = 1; k <= 4; ++k)
        for (int l = 0; l < k; ++l) T.A[k][l] = 1.0 / 6;
    for (int l = 0; l < 5; ++l) T.A[5][l] = 1.0 / 15;
    for (int k = 6; k <= 9; ++k) {
        for (int l = 0; l < 5; ++l) T.A[k][l] = 1.0 / 15;
        for (int l = 5; l < k; ++l) T.A[k][l] = 1.0 / 6;
    }
    const double c[10] = {0, 1.0 / 6, 2.0 / 6, 3.0 / 6, 4.0 / 6, 2.0 / 6, 3.0 / 6, 4.0 / 6, 5.0 / 6, 1.0};
    double Ac[10];
    for (int k = 0; k < 10; ++k) {
        T.c[k] = c[k];
        T.b[k] = 0.1;
        Ac[k] = 0.0;
        for (int l = 0; l < k; ++l) Ac[k] += T.A[k][l] * c[l];
    }
    double M[4][9];
    for (int q = 0; q < 9; ++q) {
        M[0][q] = 1.0;
        M[1][q] = c[q];
        M[2][q] = c[q] * c[q];
        M[3][q] = Ac[q];
    }
    double G[4][5];
    const double r[4] = {1.0, 0.5, 1.0 / 3, 1.0 / 6};
    for (int i = 0; i < 4; ++i) {
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
            for (int q = 0; q < 9; ++q) s += M[i][q] * M[j][q];
            G[i][j] = s;
        }
        G[i][4] = r[i];
    }
    for (int k = 0; k < 4; ++k) {  // Gauss-Jordan with partial pivoting on the 4x4 Gram system
        int p = k;
        for (int i = k + 1; i < 4; ++i)
            if (std::fabs(G[i][k]) > std::fabs(G[p][k])) p = i;
        for (int j = 0; j < 5; ++j) std::swap(G[k][j], G[p][j]);
        for (int i = 0; i < 4; ++i) {
            if (i == k) continue;
            const double f = G[i][k] / G[k][k];
            for (int j = k; j < 5; ++j) G[i][j] -= f * G[k][j];
        }
    }
    double lam[4];
    for (int i = 0; i < 4; ++i) lam[i] = G[i][4] / G[i][i];
    for (int q = 0; q < 10; ++q) {
        double bh = 0.0;
        if (q < 9)
            for (int i = 0; i < 4; ++i) bh += M[i][q] * lam[i];
        T.e[q] = T.b[q] - bh;
    }
    T.fsal = false;
    return T;
}


Layout make_layout(const dmfe_params& p) {
    Layout lo{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align_up(bytes);
        return at;
    };
    if (p.mode == DMFE_ADAPTIVE) {
        const size_t L = size_t(p.L), Mc = size_t(p.M_cap > 0 ? p.M_cap : p.L);
        // Mc history slots and the stage slot after them
        lo.hist = take((Mc + 1) * L * (p.precision == DMFE_FP32_COMP ? sizeof(HPoint32) : sizeof(HPoint)));
        lo.lhist = take(p.log_r ? (Mc + 1) * L * sizeof(LogPoint) : 0);
        lo.thist = take(Mc * sizeof(double));
        lo.slot = take(Mc * sizeof(int));
        lo.th = take(L * sizeof(double));
        lo.thc = take(L * sizeof(double));
        lo.nu = take(L * sizeof(double));
        const size_t s = size_t(p.s == 0 ? 10 : p.s);
        lo.bw = take(p.theta_interp != DMFE_INTERP_INDEX_LAGRANGE ? (L - s + 1) * (s + 1) * sizeof(double) : 0);
        lo.X = take(L * L * sizeof(double));
        lo.Xd = take(L * L * sizeof(double));
        lo.y = take(L * sizeof(YPoint));
        lo.ys = take(L * sizeof(YPoint));
        lo.ynew = take(L * sizeof(YPoint));
        lo.k = take(10 * L * sizeof(YPoint));
        lo.mue = take(2 * sizeof(double));
        lo.eps = take(sizeof(double));
        lo.diag = take(2 * sizeof(double));
        lo.eps_n = take(Mc * sizeof(double));
        lo.eps_part = take(2 * size_t(sparsify_chunks(int(L))) * Mc * sizeof(double));
        lo.obs = take(2 * Mc * sizeof(double));
        lo.rhs_y = take(L * sizeof(YPoint));
        lo.rhs_k = take(L * sizeof(YPoint));
        lo.io = take(64 * L * sizeof(double));
    } else {
        const size_t N = size_t(p.N), cap = N + 2, ntri = (N + 1) * (N + 2) / 2;
        lo.uC = take(ntri * sizeof(double));
        lo.uR = take(ntri * sizeof(double));
        lo.uE = take((N + 1) * sizeof(double));
        lo.uy0 = take(2 * cap * sizeof(double));
        lo.uy1 = take(2 * cap * sizeof(double));
        lo.uys = take(2 * cap * sizeof(double));
        lo.uk = take(4 * 2 * cap * sizeof(double));
    }
    lo.total = off;
    return lo;
}

dmfe_status validate(const dmfe_params* p) {
    if (!p) return DMFE_ERR_INVALID;
    if (p->n_terms < 1 || p->n_terms > DMFE_MAX_TERMS) return DMFE_ERR_INVALID;
    for (int k = 0; k < p->n_terms; ++k) {
        if (p->p[k] < 2 || p->p[k] > DMFE_MAX_P) return DMFE_ERR_INVALID;
        if (!(p->a2[k] >= 0.0) || !std::isfinite(p->a2[k])) return DMFE_ERR_INVALID;
    }
    if (!(p->T >= 0.0) || !std::isfinite(p->T) || !(p->beta0 >= 0.0) || !std::isfinite(p->beta0))
        return DMFE_ERR_INVALID;
    if (p->mode == DMFE_UNIFORM) {
        if (!(p->h > 0.0) || !std::isfinite(p->h) || p->N < 1 || p->N > 200000) return DMFE_ERR_INVALID;
        if (p->precision != DMFE_FP64) return DMFE_ERR_UNSUPPORTED;
        return DMFE_OK;
    }
    if (p->mode != DMFE_ADAPTIVE) return DMFE_ERR_INVALID;
    const int s = p->s == 0 ? 10 : p->s;
    if (s < 4 || s > 16 || (s & 1)) return DMFE_ERR_INVALID;
    if (p->theta_interp < DMFE_INTERP_INDEX_LAGRANGE || p->theta_interp > DMFE_INTERP_THETA_FH) return DMFE_ERR_INVALID;
    const bool fh = p->theta_interp == DMFE_INTERP_INDEX_FH || p->theta_interp == DMFE_INTERP_THETA_FH;
    if (fh && (p->fh_d < 0 || p->fh_d > s - 1)) return DMFE_ERR_INVALID;
    if (p->log_r != 0 && p->log_r != 1) return DMFE_ERR_INVALID;
    if (p->L < std::max(2 * s, 16) || p->L > 16384) return DMFE_ERR_INVALID;
    const int Mc = p->M_cap == 0 ? p->L : p->M_cap;
    // beyond the slice times that LDS holds (about 17K with the default stencil, 20K with the others),
    // the history-integral kernel reads them from global memory
    if (Mc < 16 || Mc > 65536) return DMFE_ERR_INVALID;
    if (!(p->t_max > std::exp(1.0)) || !std::isfinite(p->t_max)) return DMFE_ERR_INVALID;
    if (!(p->eps > 0.0) || !(p->dt0 > 0.0) || !(p->dt_min >= 0.0) || p->dt_min >= p->dt0) return DMFE_ERR_INVALID;
    if (p->auto_passes < 0 || p->scheme_policy < 0 || p->scheme_policy > 2) return DMFE_ERR_INVALID;
    if (p->grid_alpha != 0.0) return DMFE_ERR_UNSUPPORTED;
    if (p->precision != DMFE_FP64 && p->precision != DMFE_FP32_COMP) return DMFE_ERR_INVALID;
    return DMFE_OK;
}

Model make_model(const dmfe_params& p) {
    Model m{};
    m.T = p.T;
    m.beta0 = p.beta0;
    m.pmax = 2;
    for (int k = 0; k < p.n_terms; ++k) {
        const int q = p.p[k];
        const double a2 = p.a2[k];
        m.fc[q] += 0.5 * a2;
        m.f1[q - 1] += 0.5 * a2 * q;
        m.f2[q - 2] += 0.5 * a2 * q * (q - 1);
        m.pmax = std::max(m.pmax, q);
    }
    return m;
}

double f2_at_one(const Model& m) {
    double s = 0.0;
    for (int k = 0; k < PCAP; ++k) s += m.f2[k];
    return s;
}



dmfe_status fail(hipError_t e, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return DMFE_ERR_DEVICE;
}
dmfe_status fail_msg(dmfe_status s, const std::string& msg) {
    set_error(msg);
    return s;
}

// Event pair around one launch when timing is on; nullptr otherwise.
dmfe_handle::EvPair* timing_begin(dmfe_handle* h, int kernel, int64_t slices) {
    if (!h->timing || !((h->timing_mask >> kernel) & 1u)) return nullptr;
    dmfe_handle::EvPair p;
    if (!h->ev_pool.empty()) {
        p = h->ev_pool.back();
        h->ev_pool.pop_back();
    } else if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) {
        return nullptr;
    }
    p.kernel = kernel;
    p.slices = slices;
    if (hipEventRecord(p.a, h->stream) != hipSuccess) {
        h->ev_pool.push_back(p);
        return nullptr;
    }
    h->ev_pending.push_back(p);
    return &h->ev_pending.back();
}
void timing_end(dmfe_handle* h, dmfe_handle::EvPair* p) {
    if (p) (void)hipEventRecord(p->b, h->stream);
}
// Accumulate finished event pairs (the stream has been synchronised).
void timing_drain(dmfe_handle* h) {
    for (auto& p : h->ev_pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            h->kt_launches[p.kernel] += 1;
            h->kt_ms[p.kernel] += ms;
            h->kt_slices[p.kernel] += p.slices;
        }
        h->ev_pool.push_back(p);
    }
    h->ev_pending.clear();
}

StageBufs handle_bufs(const dmfe_handle* h) {
    StageBufs b{};
    b.stage = stage_slot(h);
    LogPoint* lm = log_mirror(h);
    b.lstage = lm ? lm + size_t(h->Mc) * h->L : nullptr;
    b.mue = h->at<double>(h->lo.mue);
    b.diag = h->at<double>(h->lo.diag);
    return b;
}

StageArgs stage_args(const dmfe_handle* h, double t, int nb, const YPoint* y, YPoint* kout, void* store) {
    return stage_args(h, t, nb, y, kout, store, handle_bufs(h));
}

StageArgs stage_args(const dmfe_handle* h, double t, int nb, const YPoint* y, YPoint* kout, void* store,
                     const StageBufs& b) {
    StageArgs a{};
    a.L = h->L;
    a.nb = nb;
    a.t = t;
    a.tb = nb > 0 ? h->thist[nb - 1] : 0.0;
    a.X = h->at<double>(h->lo.X);
    a.Xd = h->at<double>(h->lo.Xd);
    a.th = h->at<double>(h->lo.th);
    a.thc = h->at<double>(h->lo.thc);
    a.nu = h->at<double>(h->lo.nu);
    a.thist = h->at<double>(h->lo.thist);
    a.slot = h->at<int>(h->lo.slot);
    a.hist = h->at<void>(h->lo.hist);
    a.stage = b.stage;
    a.fp32 = h->fp32;
    a.y = y;
    a.mue = b.mue;
    a.kout = kout;
    a.store = store;
    a.diag = b.diag;
    a.interp = h->p.theta_interp;
    a.log_r = h->p.log_r;
    a.bw = h->at<double>(h->lo.bw);
    for (int k = 0; k < 16; ++k) a.fh_c[k] = h->fh_c[k];
    a.lhist = log_mirror(h);
    a.lstage = b.lstage;
    a.m = h->m;
    return a;
}

LogPoint* log_mirror(const dmfe_handle* h) { return h->p.log_r ? h->at<LogPoint>(h->lo.lhist) : nullptr; }

dmfe_status rebuild_log_mirror(dmfe_handle* h) {
    if (!h->p.log_r) return DMFE_OK;
    HCHK(launch_log_mirror(h->L, h->M, h->at<int>(h->lo.slot), h->at<void>(h->lo.hist), h->fp32, log_mirror(h),
                           h->stream));
    return DMFE_OK;
}

// one right-hand-side evaluation: mu(t) then the history integrals
dmfe_status eval_rhs(dmfe_handle* h, double t, int nb, const YPoint* y, YPoint* kout, void* store,
                     const StageBufs& b, bool timed) {
    auto* e1 = timed ? timing_begin(h, DMFE_K_STAGE_PREP, 0) : nullptr;
    HCHK(launch_stage_prep(h->m, h->L, t, h->at<double>(h->lo.nu), y, b.mue, b.stage, h->fp32, b.lstage,
                           h->stream));
    timing_end(h, e1);
    auto* e2 = timed ? timing_begin(h, DMFE_K_HIST_INTEGRAL, nb) : nullptr;
    HCHK(launch_hist_integral(stage_args(h, t, nb, y, kout, store, b), h->s, h->stream));
    timing_end(h, e2);
    h->rhs_evals += 1;
    return DMFE_OK;
}

dmfe_status eval_rhs(dmfe_handle* h, double t, int nb, const YPoint* y, YPoint* kout, void* store) {
    return eval_rhs(h, t, nb, y, kout, store, handle_bufs(h), true);
}

size_t point_bytes(const dmfe_handle* h) { return h->fp32 ? sizeof(HPoint32) : sizeof(HPoint); }
void* slot_ptr(dmfe_handle* h, int slot) {
    return h->at<char>(h->lo.hist) + size_t(slot) * h->L * point_bytes(h);
}
void* stage_slot(const dmfe_handle* h) {
    return const_cast<dmfe_handle*>(h)->at<char>(h->lo.hist) + size_t(h->Mc) * h->L * point_bytes(h);
}

dmfe_status upload_order(dmfe_handle* h) {
    HCHK(hipMemcpyAsync(h->at<double>(h->lo.thist), h->thist.data(), sizeof(double) * h->M, hipMemcpyHostToDevice,
                        h->stream));
    HCHK(hipMemcpyAsync(h->at<int>(h->lo.slot), h->slot.data(), sizeof(int) * h->M, hipMemcpyHostToDevice,
                        h->stream));
    // the host vectors may change before the copies run: finish them here
    HCHK(hipStreamSynchronize(h->stream));
    return DMFE_OK;
}

dmfe_status sparsify_pass(dmfe_handle* h, int64_t* removed_out) {
    *removed_out = 0;
    const int M = h->M;
    if (M < 13) return DMFE_OK;
    const int count = M - 12;  // candidates 1..M-12
    double* eps_n = h->at<double>(h->lo.eps_n);
    auto* ev = timing_begin(h, DMFE_K_SPARSIFY, 0);
    HCHK(launch_sparsify_residual(h->L, 1, count, h->at<double>(h->lo.thist), h->at<int>(h->lo.slot),
                                  h->at<void>(h->lo.hist), h->fp32, eps_n, h->at<double>(h->lo.eps_part), h->Mc,
                                  h->stream));
    timing_end(h, ev);
    std::vector<double> e(M, -1.0);
    HCHK(hipMemcpyAsync(e.data() + 1, eps_n + 1, sizeof(double) * count, hipMemcpyDeviceToHost, h->stream));
    HCHK(hipStreamSynchronize(h->stream));
    std::vector<uint8_t> drop(M, 0);
    int64_t nrem = 0;
    dmfe_sparsify_select(e.data(), M, M - 12, h->p.eps / 10.0, drop.data(), &nrem);
    if (nrem > 0) {
        int w = 0;
        for (int n = 0; n < M; ++n) {
            if (drop[n]) {
                h->free_slots.push_back(h->slot[n]);
                continue;
            }
            h->thist[w] = h->thist[n];
            h->slot[w] = h->slot[n];
            ++w;
        }
        // only the first M-12 slices are candidates, so the slices without a stored
        // d/dt (at most the newest) are still the last ones
        h->nb_valid = w - (M - h->nb_valid);
        h->M = w;
        h->thist.resize(w);
        h->slot.resize(w);
        dmfe_status st = upload_order(h);
        if (st != DMFE_OK) return st;
        h->fsal_valid = false;
    }
    h->n_sparsify += 1;
    h->removed += nrem;
    *removed_out = nrem;
    return DMFE_OK;
}

void fill_info(const dmfe_handle* h, dmfe_step_info* info) {
    if (!info) return;
    std::memset(info, 0, sizeof(*info));
    info->accepted = h->accepted;
    info->rejected = h->rejected;
    info->reverts = h->reverts;
    info->sparsify_calls = h->n_sparsify;
    info->removed = h->removed;
    info->rhs_evals = h->rhs_evals;
    info->scheme = h->scheme;
    info->eps_rk = h->eps_rk;
    info->nb_valid = h->p.mode == DMFE_UNIFORM ? int32_t(h->un + 1) : h->nb_valid;
    if (h->p.mode == DMFE_UNIFORM) {
        info->M = h->un + 1;
        info->t = double(h->un) * h->p.h;
        info->dt = h->p.h;
    } else {
        info->M = h->M;
        info->t = h->t;
        info->dt = h->dt;
    }
}

// ------------------------------------------------------------------ adaptive stepping
dmfe_status step_begin(dmfe_handle* h) {
    if (h->M >= h->Mc) {
        int64_t got = 0;
        const int passes = h->p.auto_passes > 0 ? h->p.auto_passes : 1;
        for (int q = 0; q < passes; ++q) {
            int64_t r = 0;
            const dmfe_status st = sparsify_pass(h, &r);
            if (st != DMFE_OK) return st;
            got += r;
        }
        if (got == 0) return DMFE_ERR_CAPACITY;
    }
    auto& c = h->cur;
    c.T = h->scheme == DMFE_SCHEME_DP5 ? &h->dp5 : &h->ssp;
    c.M = h->M;
    c.dt = h->dt;
    c.tn = h->thist[h->M - 1];
    c.next_slot = h->free_slots.back();
    c.st = 0;
    c.active = 1;
    return DMFE_OK;
}

dmfe_status step_stage(dmfe_handle* h) {
    auto& c = h->cur;
    const Tableau& T = *c.T;
    const int L = h->L, st = c.st;
    YPoint* y0 = h->at<YPoint>(h->lo.y);
    YPoint* ys = h->at<YPoint>(h->lo.ys);
    YPoint* kb = h->at<YPoint>(h->lo.k);
    YPoint* kst = kb + size_t(st) * L;
    const double tst = c.tn + T.c[st] * c.dt;
    if (st == 0) {
        // first-same-as-last: k_0 already holds the last step's final stage (written on accept)
        if (!h->fsal_valid) {
            const dmfe_status s = eval_rhs(h, tst, c.M - 1, y0, kst, slot_ptr(h, h->slot[c.M - 1]));
            if (s != DMFE_OK) return s;
        }
    } else {
        auto* ev = timing_begin(h, DMFE_K_RK, 0);
        HCHK(launch_rk_combine(L, y0, kb, st, T.A[st], c.dt, ys, h->stream));
        timing_end(h, ev);
        // the last DP5 stage is F(t + dt, y_new): it is also the stored d/dt of the next slice
        void* store = (T.fsal && st == T.S - 1) ? slot_ptr(h, c.next_slot) : nullptr;
        const dmfe_status s = eval_rhs(h, tst, c.M, ys, kst, store);
        if (s != DMFE_OK) return s;
    }
    c.st = st + 1;
    return DMFE_OK;
}

dmfe_status step_finish(dmfe_handle* h) {
    auto& c = h->cur;
    const Tableau& T = *c.T;
    auto* evf = timing_begin(h, DMFE_K_RK, 0);
    HCHK(launch_rk_finish(h->L, h->at<YPoint>(h->lo.y), h->at<YPoint>(h->lo.k), T.S, T.b, T.e, c.dt,
                          h->at<YPoint>(h->lo.ynew), h->at<double>(h->lo.eps), h->stream));
    timing_end(h, evf);
    HCHK(hipMemcpyAsync(h->pinned, h->at<double>(h->lo.eps), sizeof(double), hipMemcpyDeviceToHost, h->stream));
    return DMFE_OK;
}

dmfe_status step_decide(dmfe_handle* h, double err) {
    auto& c = h->cur;
    const Tableau& T = *c.T;
    const int L = h->L, M = c.M;
    const double dt = c.dt, tn = c.tn;
    c.active = 0;
    h->nb_valid = M;
    h->eps_rk = err;
    dmfe_control ctl{};
    ctl.eps = h->p.eps;
    ctl.dt = dt;
    ctl.dt_min = h->p.dt_min;
    ctl.rho = 4.0 * std::sqrt(f2_at_one(h->m));
    ctl.M = M;
    ctl.scheme = h->scheme;
    ctl.policy = h->p.scheme_policy;
    int32_t acc = 0, nrev = 0;
    const dmfe_status cs = dmfe_control_update(&ctl, err, &acc, &nrev);
    if (cs == DMFE_ERR_NONFINITE) return cs;
    YPoint* y0 = h->at<YPoint>(h->lo.y);
    if (acc) {
        const int slot = c.next_slot;
        h->free_slots.pop_back();
        LogPoint* lm = log_mirror(h);
        h->thist.push_back(tn + dt);
        h->slot.push_back(slot);
        h->M = M + 1;
        h->nb_valid = T.fsal ? h->M : M;
        h->t = tn + dt;
        // one launch: the new slice, the new state, the next step's first stage, and the new
        // slice's time and slot in the device index arrays
        YPoint* kb = h->at<YPoint>(h->lo.k);
        AcceptArgs aa{};
        aa.L = L;
        aa.M = M;
        aa.slot_new = slot;
        aa.t_new = h->t;
        aa.ynew = h->at<YPoint>(h->lo.ynew);
        aa.slot_dst = slot_ptr(h, slot);
        aa.lslot = lm ? lm + size_t(slot) * L : nullptr;
        aa.y0 = y0;
        aa.k_last = T.fsal ? kb + size_t(T.S - 1) * L : nullptr;
        aa.k_first = T.fsal ? kb : nullptr;
        aa.thist = h->at<double>(h->lo.thist);
        aa.slots = h->at<int>(h->lo.slot);
        HCHK(launch_accept(aa, h->fp32, h->stream));
        h->fsal_valid = T.fsal;
        h->accepted += 1;
    } else {
        for (int q = 0; q < nrev; ++q) {
            h->free_slots.push_back(h->slot.back());
            h->slot.pop_back();
            h->thist.pop_back();
        }
        h->M = M - nrev;
        h->nb_valid = std::min(h->nb_valid, h->M);
        h->t = h->thist[h->M - 1];
        HCHK(launch_load_state(L, slot_ptr(h, h->slot[h->M - 1]), h->fp32, y0, h->stream));
        h->fsal_valid = false;
        h->rejected += 1;
        h->reverts += nrev;
    }
    h->dt = ctl.dt;
    h->scheme = ctl.scheme;
    return cs;
}

dmfe_status adaptive_step_once(dmfe_handle* h) {
    dmfe_status st = step_begin(h);
    if (st != DMFE_OK) return st;
    while (h->cur.st < h->cur.T->S) {
        st = step_stage(h);
        if (st != DMFE_OK) return st;
    }
    st = step_finish(h);
    if (st != DMFE_OK) return st;
    HCHK(hipStreamSynchronize(h->stream));
    timing_drain(h);
    return step_decide(h, h->pinned[0]);
}

dmfe_status adaptive_step(dmfe_handle* h, double t_target, int64_t max_steps) {
    for (int64_t k = 0; k < max_steps; ++k) {
        if (h->t >= t_target || h->t >= h->p.t_max) break;
        const dmfe_status st = adaptive_step_once(h);
        if (st != DMFE_OK) return st;
    }
    return h->t >= h->p.t_max ? DMFE_DONE : DMFE_OK;
}

// ------------------------------------------------------------------ uniform stepping
dmfe_status uniform_step(dmfe_handle* h, double t_target, int64_t max_steps) {
    const int64_t N = h->p.N;
    const double hh = h->p.h;
    const int cap = int(N + 2);
    double* C = h->at<double>(h->lo.uC);
    double* R = h->at<double>(h->lo.uR);
    double* E = h->at<double>(h->lo.uE);
    double* ys = h->at<double>(h->lo.uys);
    double* k = h->at<double>(h->lo.uk);
    double* kk[4] = {k, k + 2 * cap, k + 4 * cap, k + 6 * cap};
    const double offs[4] = {0.0, 0.5 * hh, 0.5 * hh, hh};
    for (int64_t s = 0; s < max_steps && h->un < N; ++s) {
        if (double(h->un) * hh >= t_target) break;
        const int n = int(h->un);
        double* y0 = h->at<double>(h->ucur ? h->lo.uy1 : h->lo.uy0);
        double* y1 = h->at<double>(h->ucur ? h->lo.uy0 : h->lo.uy1);
        for (int st = 0; st < 4; ++st) {
            const double* ycur = y0;
            if (st > 0) {
                HCHK(launch_uniform_axpy(n + 1, cap, y0, kk[st - 1], offs[st], ys, h->stream));
                ycur = ys;
            }
            UniArgs a{};
            a.n = n;
            a.h = hh;
            a.delta = offs[st];
            a.C = C;
            a.R = R;
            a.y = ycur;
            a.cap = cap;
            a.kout = kk[st];
            a.m = h->m;
            HCHK(launch_uniform_rhs(a, h->stream));
            h->rhs_evals += 1;
        }
        HCHK(launch_uniform_rk4_append(n, cap, hh, y0, kk[0], kk[1], kk[2], kk[3], C, R, y1, h->stream));
        HCHK(launch_uniform_energy(h->m, n + 1, hh, C, R, E, h->stream));
        h->ucur ^= 1;
        h->un += 1;
        h->accepted += 1;
    }
    HCHK(hipStreamSynchronize(h->stream));
    return h->un >= N ? DMFE_DONE : DMFE_OK;
}

}  // namespace core
}  // namespace dmfe

using namespace dmfe;
using namespace dmfe::core;

extern "C" {

const char* dmfe_status_string(dmfe_status s) {
    switch (s) {
    case DMFE_OK: return "ok";
    case DMFE_DONE: return "done: t reached t_max";
    case DMFE_ERR_INVALID: return "invalid parameters or arguments";
    case DMFE_ERR_NOMEM: return "out of memory or workspace too small";
    case DMFE_ERR_CAPACITY: return "history full and sparsification freed nothing";
    case DMFE_ERR_STEP_UNDERFLOW: return "step size below dt_min";
    case DMFE_ERR_NONFINITE: return "non-finite error estimate";
    case DMFE_ERR_DEVICE: return "HIP error";
    case DMFE_ERR_UNSUPPORTED: return "not supported";
    case DMFE_ERR_BUFFER: return "destination buffer too small";
    default: return "unknown status";
    }
}

const char* dmfe_last_error(void) { return last_error(); }

dmfe_status dmfe_param_record(const dmfe_handle* h, char* buf, size_t cap, size_t* needed) {
    if (!h) return DMFE_ERR_INVALID;
    std::string out;
    char line[512];
    auto put = [&](const char* key, const std::string& val) {
        std::snprintf(line, sizeof(line), "%s = %s\n", key, val.c_str());
        out += line;
    };
    auto num = [](double v) {
        char b[40];
        std::snprintf(b, sizeof(b), "%.17g", v);
        return std::string(b);
    };
    auto inum = [](long long v) { return std::to_string(v); };
    const dmfe_params& p = h->p;
    out += "# DMFE solve: parameter record\n";
#ifdef DMFE_SOURCE_REVISION
    put("library_revision", DMFE_SOURCE_REVISION);
#else
    put("library_revision", "unknown");
#endif
    put("compiler", __VERSION__);
    int rt = 0;
    put("hip_runtime", hipRuntimeGetVersion(&rt) == hipSuccess ? inum(rt) : "unknown");
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) {
        put("device", std::to_string(h->device) + " " + prop.name + " (" + prop.gcnArchName + "), " +
                          inum(prop.multiProcessorCount) + " CUs, " + num(double(prop.totalGlobalMem) / 1073741824.0) +
                          " GiB");
    }
    {  // the process command line, arguments separated by spaces
        std::string cmd;
        if (FILE* f = std::fopen("/proc/self/cmdline", "rb")) {
            int c;
            while ((c = std::fgetc(f)) != EOF && cmd.size() < 400) cmd += c == 0 ? ' ' : char(c);
            std::fclose(f);
        }
        while (!cmd.empty() && cmd.back() == ' ') cmd.pop_back();
        put("command_line", cmd.empty() ? "unknown" : cmd);
    }
    put("mode", p.mode == DMFE_ADAPTIVE ? "adaptive" : "uniform");
    std::string model;
    for (int k = 0; k < p.n_terms; ++k) model += (k ? " + " : "") + num(p.a2[k]) + " q^" + inum(p.p[k]) + "/2";
    put("f(q)", model);
    put("T", num(p.T));
    put("beta0", num(p.beta0));
    put("precision", p.precision == DMFE_FP32_COMP ? "fp32-comp" : "fp64");
    if (p.mode == DMFE_UNIFORM) {
        put("h", num(p.h));
        put("N", inum(p.N));
    } else {
        static const char* schemes[] = {"index-lagrange", "theta-lagrange", "index-floater-hormann",
                                        "theta-floater-hormann"};
        put("t_max", num(p.t_max));
        put("grid_gamma", num(h->gamma));
        put("grid_alpha", num(p.grid_alpha));
        put("grid_delta", num(p.grid_delta));
        put("L", inum(p.L));
        put("M_cap", inum(h->Mc));
        put("eps", num(p.eps));
        put("dt0", num(p.dt0));
        put("dt_min", num(p.dt_min));
        put("s", inum(h->s));
        put("theta_interp", schemes[p.theta_interp]);
        if (p.theta_interp == DMFE_INTERP_INDEX_FH || p.theta_interp == DMFE_INTERP_THETA_FH) put("fh_d", inum(p.fh_d));
        put("log_r", inum(p.log_r));
        put("auto_passes", inum(p.auto_passes));
        put("scheme_policy", inum(p.scheme_policy));
    }
    dmfe_step_info info{};
    fill_info(h, &info);
    put("state_t", num(info.t));
    put("state_dt", num(info.dt));
    put("state_M", inum(info.M));
    put("state_scheme", info.scheme == DMFE_SCHEME_SSPRK104 ? "ssprk104" : "dp5");
    put("accepted", inum(info.accepted));
    put("rejected", inum(info.rejected));
    put("reverts", inum(info.reverts));
    put("sparsify_calls", inum(info.sparsify_calls));
    put("removed", inum(info.removed));
    put("rhs_evals", inum(info.rhs_evals));
    if (needed) *needed = out.size() + 1;
    if (cap < out.size() + 1) return DMFE_ERR_BUFFER;
    std::memcpy(buf, out.c_str(), out.size() + 1);
    return DMFE_OK;
}

dmfe_status dmfe_footprint(const dmfe_params* params, size_t* bytes) {
    const dmfe_status v = validate(params);
    if (v != DMFE_OK) return v;
    if (!bytes) return DMFE_ERR_INVALID;
    *bytes = make_layout(*params).total;
    return DMFE_OK;
}

dmfe_status dmfe_grid(const dmfe_params* params, double* theta, double* theta_c, double* nu, double* gamma) {
    const dmfe_status v = validate(params);
    if (v != DMFE_OK) return v;
    if (params->mode != DMFE_ADAPTIVE) return DMFE_ERR_INVALID;
    const int L = params->L;
    std::vector<double> th(L), thc(L), w(L);
    const double g = lambert_gamma(params->t_max);
    theta_grid(L, g, th.data(), thc.data());
    if (quintic_weights(L, th.data(), w.data()) != 0) return DMFE_ERR_INVALID;
    if (theta) std::memcpy(theta, th.data(), sizeof(double) * L);
    if (theta_c) std::memcpy(theta_c, thc.data(), sizeof(double) * L);
    if (nu) std::memcpy(nu, w.data(), sizeof(double) * L);
    if (gamma) *gamma = g;
    return DMFE_OK;
}

dmfe_status dmfe_control_update(dmfe_control* st, double eps_rk, int32_t* accepted, int32_t* n_revert) {
    if (!st || !accepted || !n_revert) return DMFE_ERR_INVALID;
    *accepted = 0;
    *n_revert = 0;
    if (!std::isfinite(eps_rk)) return DMFE_ERR_NONFINITE;
    double dt = st->dt;
    if (eps_rk > 2.0 * st->eps) {
        *n_revert = int32_t(std::min<int64_t>(10, std::max<int64_t>(st->M - 1, 0)));
        dt = 0.5 * dt;
    } else {
        *accepted = 1;
        if (eps_rk > st->eps) dt = 0.9 * dt;
        else if (eps_rk < 0.5 * st->eps) dt = 1.01 * dt;
        if (st->scheme == DMFE_SCHEME_DP5 && st->policy == 0 && dt * st->rho >= kDp5Limit) {
            st->scheme = DMFE_SCHEME_SSPRK104;
            dt = 0.5 * dt;
        }
        if (st->scheme == DMFE_SCHEME_SSPRK104 && dt * st->rho > kSspLimit) dt = kSspLimit / st->rho;
    }
    st->dt = dt;
    if (dt < st->dt_min) return DMFE_ERR_STEP_UNDERFLOW;
    return DMFE_OK;
}

dmfe_status dmfe_sparsify_select(const double* eps_n, int64_t M, int64_t last, double thr, uint8_t* drop,
                                 int64_t* removed) {
    if (!eps_n || !drop || M < 0 || last >= M) return DMFE_ERR_INVALID;
    for (int64_t n = 0; n < M; ++n) drop[n] = 0;
    int64_t cnt = 0;
    for (int64_t n = 1; n <= last;) {
        if (eps_n[n] < thr) {
            drop[n] = 1;
            ++cnt;
            n += 2;
        } else {
            n += 1;
        }
    }
    if (removed) *removed = cnt;
    return DMFE_OK;
}

dmfe_status dmfe_create(const dmfe_params* params, const dmfe_resources* res, dmfe_handle** out) {
    if (!out) return DMFE_ERR_INVALID;
    *out = nullptr;
    const dmfe_status v = validate(params);
    if (v != DMFE_OK) return v;
    dmfe_handle* h = new (std::nothrow) dmfe_handle();
    if (!h) return DMFE_ERR_NOMEM;
    h->p = *params;
    if (h->p.mode == DMFE_ADAPTIVE) {
        if (h->p.s == 0) h->p.s = 10;
        if (h->p.M_cap == 0) h->p.M_cap = h->p.L;
        if (h->p.auto_passes == 0) h->p.auto_passes = 1;
    }
    h->lo = make_layout(h->p);
    h->device = res ? res->device : 0;
    h->stream = res ? reinterpret_cast<hipStream_t>(res->stream) : nullptr;
    h->m = make_model(h->p);
    auto bail = [&](dmfe_status s) {
        dmfe_destroy(h);
        return s;
    };
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return bail(fail(e, "hipSetDevice"));
    if (res && res->workspace) {
        if (res->workspace_bytes < h->lo.total) return bail(DMFE_ERR_NOMEM);
        h->base = reinterpret_cast<char*>(res->workspace);
        h->owns = false;
    } else {
        e = hipMalloc(reinterpret_cast<void**>(&h->base), h->lo.total);
        if (e != hipSuccess) {
            h->base = nullptr;
            set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
            return bail(DMFE_ERR_NOMEM);
        }
        h->owns = true;
    }
    e = hipHostMalloc(reinterpret_cast<void**>(&h->pinned), 64 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) return bail(fail(e, "hipHostMalloc"));

    if (h->p.mode == DMFE_UNIFORM) {
        const int64_t N = h->p.N;
        const int cap = int(N + 2);
        const double one = 1.0;
        e = hipMemsetAsync(h->base, 0, h->lo.total, h->stream);
        if (e != hipSuccess) return bail(fail(e, "hipMemsetAsync"));
        std::vector<double> y(2 * cap, 0.0);
        y[0] = 1.0;
        y[cap] = 1.0;
        if ((e = hipMemcpyAsync(h->at<double>(h->lo.uC), &one, sizeof(double), hipMemcpyHostToDevice, h->stream)) ||
            (e = hipMemcpyAsync(h->at<double>(h->lo.uR), &one, sizeof(double), hipMemcpyHostToDevice, h->stream)) ||
            (e = hipMemcpyAsync(h->at<double>(h->lo.uy0), y.data(), sizeof(double) * 2 * cap, hipMemcpyHostToDevice,
                                h->stream)))
            return bail(fail(e, "hipMemcpyAsync"));
        e = launch_uniform_energy(h->m, 0, h->p.h, h->at<double>(h->lo.uC), h->at<double>(h->lo.uR),
                                  h->at<double>(h->lo.uE), h->stream);
        if (e != hipSuccess) return bail(fail(e, "uniform energy"));
        e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return bail(fail(e, "hipStreamSynchronize"));
        h->un = 0;
        *out = h;
        return DMFE_OK;
    }

    // adaptive: run-constant grid data
    h->L = h->p.L;
    h->s = h->p.s;
    h->Mc = h->p.M_cap;
    h->fp32 = h->p.precision == DMFE_FP32_COMP ? 1 : 0;
    const int L = h->L;
    h->th.resize(L);
    h->thc.resize(L);
    h->nu.resize(L);
    h->gamma = lambert_gamma(h->p.t_max);
    theta_grid(L, h->gamma, h->th.data(), h->thc.data());
    if (quintic_weights(L, h->th.data(), h->nu.data()) != 0) return bail(DMFE_ERR_INVALID);
    h->Dg = std::atan(std::sinh(h->gamma));
    h->xscale = double(L - 1) / (2.0 * h->gamma);
    h->eg = std::exp(h->gamma);
    h->egi = std::exp(-h->gamma);
    h->dp5 = make_dp5();
    h->ssp = make_ssprk104();
    h->scheme = h->p.scheme_policy == 1 ? DMFE_SCHEME_SSPRK104 : DMFE_SCHEME_DP5;
    h->dt = h->p.dt0;
    if ((e = hipMemcpyAsync(h->at<double>(h->lo.th), h->th.data(), sizeof(double) * L, hipMemcpyHostToDevice,
                            h->stream)) ||
        (e = hipMemcpyAsync(h->at<double>(h->lo.thc), h->thc.data(), sizeof(double) * L, hipMemcpyHostToDevice,
                            h->stream)) ||
        (e = hipMemcpyAsync(h->at<double>(h->lo.nu), h->nu.data(), sizeof(double) * L, hipMemcpyHostToDevice,
                            h->stream)))
        return bail(fail(e, "hipMemcpyAsync"));
    if (h->p.theta_interp != DMFE_INTERP_INDEX_LAGRANGE) {
        std::vector<double> bw(size_t(L - h->s + 1) * (h->s + 1));
        stencil_coefficients(L, h->s, h->p.theta_interp, h->p.fh_d, h->th.data(), h->thc.data(), bw.data());
        for (int k = 0; k < h->s; ++k) h->fh_c[k] = bw[k];
        // synchronous: the host table goes out of scope below
        if ((e = hipMemcpyAsync(h->at<double>(h->lo.bw), bw.data(), sizeof(double) * bw.size(),
                                hipMemcpyHostToDevice, h->stream)) != hipSuccess ||
            (e = hipStreamSynchronize(h->stream)) != hipSuccess)
            return bail(fail(e, "hipMemcpyAsync"));
    }
    {
        GridArgs g{};
        g.L = L;
        g.xscale = h->xscale;
        g.eg = h->eg;
        g.egi = h->egi;
        g.Dg = h->Dg;
        g.th = h->at<double>(h->lo.th);
        g.thc = h->at<double>(h->lo.thc);
        g.X = h->at<double>(h->lo.X);
        g.Xd = h->at<double>(h->lo.Xd);
        e = launch_coords(g, h->stream);
        if (e != hipSuccess) return bail(fail(e, "coordinate precompute"));
    }
    // initial slice t = 0: C = R = 1 (derivative filled at the first stage)
    std::vector<HPoint> s0(L, HPoint{1.0, 1.0, 0.0, 0.0});
    std::vector<HPoint32> s032(L, HPoint32{1.0f, 1.0f, 0.0f, 0.0f});
    std::vector<YPoint> y0(L, YPoint{1.0, 1.0});
    h->free_slots.clear();
    for (int q = h->Mc - 1; q >= 1; --q) h->free_slots.push_back(q);
    h->thist.assign(1, 0.0);
    h->slot.assign(1, 0);
    h->M = 1;
    h->nb_valid = 0;
    h->t = 0.0;
    if ((e = hipMemcpyAsync(slot_ptr(h, 0), h->fp32 ? static_cast<const void*>(s032.data()) : s0.data(),
                            point_bytes(h) * L, hipMemcpyHostToDevice, h->stream)) ||
        (e = hipMemcpyAsync(h->at<YPoint>(h->lo.y), y0.data(), sizeof(YPoint) * L, hipMemcpyHostToDevice,
                            h->stream)))
        return bail(fail(e, "hipMemcpyAsync"));
    dmfe_status us = upload_order(h);
    if (us == DMFE_OK) us = rebuild_log_mirror(h);
    if (us != DMFE_OK) return bail(us);
    *out = h;
    return DMFE_OK;
}

void dmfe_destroy(dmfe_handle* h) {
    if (!h) return;
    ckpt_release(h);
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    if (h->owns && h->base) (void)hipFree(h->base);
    if (h->pinned) (void)hipHostFree(h->pinned);
    for (auto* v : {&h->ev_pool, &h->ev_pending})
        for (auto& p : *v) {
            if (p.a) (void)hipEventDestroy(p.a);
            if (p.b) (void)hipEventDestroy(p.b);
        }
    delete h;
}

dmfe_status dmfe_step(dmfe_handle* h, double t_target, int64_t max_steps, dmfe_step_info* info) {
    if (!h || max_steps < 0) return DMFE_ERR_INVALID;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return fail(e, "hipSetDevice");
    const dmfe_status st = h->p.mode == DMFE_UNIFORM ? uniform_step(h, t_target, max_steps)
                                                     : adaptive_step(h, t_target, max_steps);
    fill_info(h, info);
    return st;
}

dmfe_status dmfe_get_info(dmfe_handle* h, dmfe_step_info* info) {
    if (!h || !info) return DMFE_ERR_INVALID;
    fill_info(h, info);
    return DMFE_OK;
}

dmfe_status dmfe_sparsify(dmfe_handle* h, int32_t passes, int64_t* removed) {
    if (!h || passes < 0) return DMFE_ERR_INVALID;
    if (h->p.mode != DMFE_ADAPTIVE) return DMFE_ERR_INVALID;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return fail(e, "hipSetDevice");
    int64_t tot = 0;
    for (int q = 0; q < passes; ++q) {
        int64_t r = 0;
        const dmfe_status st = sparsify_pass(h, &r);
        if (st != DMFE_OK) return st;
        tot += r;
    }
    if (removed) *removed = tot;
    return DMFE_OK;
}

dmfe_status dmfe_set_history(dmfe_handle* h, int64_t M, int64_t nb, const double* t_hist, const double* C,
                             const double* R, const double* dC, const double* dR, int32_t src_on_device, double dt,
                             int32_t scheme) {
    if (!h || h->p.mode != DMFE_ADAPTIVE) return DMFE_ERR_INVALID;
    if (M < 1 || M > h->Mc || nb < M - 1 || nb > M || !t_hist || !C || !R || !dC || !dR) return DMFE_ERR_INVALID;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return fail(e, "hipSetDevice");
    std::vector<double> th(M);
    if (src_on_device) {
        HCHK(hipMemcpy(th.data(), t_hist, sizeof(double) * M, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(th.data(), t_hist, sizeof(double) * M);
    }
    if (th[0] != 0.0) return DMFE_ERR_INVALID;
    for (int64_t n = 1; n < M; ++n)
        if (!(th[n] > th[n - 1])) return DMFE_ERR_INVALID;
    const int L = h->L;
    h->thist = th;
    h->slot.resize(M);
    for (int n = 0; n < M; ++n) h->slot[n] = n;
    h->free_slots.clear();
    for (int q = h->Mc - 1; q >= int(M); --q) h->free_slots.push_back(q);
    h->M = int(M);
    dmfe_status st = upload_order(h);
    if (st != DMFE_OK) return st;
    if (src_on_device) {
        HCHK(launch_unpack_history(L, int(M), C, R, dC, dR, h->at<int>(h->lo.slot), h->at<void>(h->lo.hist), h->fp32,
                                   h->stream));
    } else if (h->fp32) {
        std::vector<HPoint32> buf(size_t(M) * L);
        for (size_t q = 0; q < buf.size(); ++q)
            buf[q] = HPoint32{float(C[q]), float(R[q]), float(dC[q]), float(dR[q])};
        HCHK(hipMemcpyAsync(h->at<void>(h->lo.hist), buf.data(), sizeof(HPoint32) * buf.size(),
                            hipMemcpyHostToDevice, h->stream));
        HCHK(hipStreamSynchronize(h->stream));
    } else {
        std::vector<HPoint> buf(size_t(M) * L);
        for (size_t q = 0; q < buf.size(); ++q) buf[q] = HPoint{C[q], R[q], dC[q], dR[q]};
        HCHK(hipMemcpyAsync(h->at<void>(h->lo.hist), buf.data(), sizeof(HPoint) * buf.size(),
                            hipMemcpyHostToDevice, h->stream));
        HCHK(hipStreamSynchronize(h->stream));
    }
    const dmfe_status ms = rebuild_log_mirror(h);
    if (ms != DMFE_OK) return ms;
    HCHK(launch_load_state(L, slot_ptr(h, h->slot[M - 1]), h->fp32, h->at<YPoint>(h->lo.y), h->stream));
    HCHK(hipStreamSynchronize(h->stream));
    h->nb_valid = int(nb);
    h->t = th[M - 1];
    if (dt > 0.0) h->dt = dt;
    if (scheme == DMFE_SCHEME_DP5 || scheme == DMFE_SCHEME_SSPRK104) h->scheme = scheme;
    h->fsal_valid = false;
    return DMFE_OK;
}

dmfe_status dmfe_rhs(dmfe_handle* h, double t, const double* yC, const double* yR, int64_t nb, double* outC,
                     double* outR, double* mu, double* diag) {
    if (!h || h->p.mode != DMFE_ADAPTIVE || !yC || !yR || !outC || !outR) return DMFE_ERR_INVALID;
    if (nb < 0 || nb > h->M) return DMFE_ERR_INVALID;
    if (nb > 0 && !(t >= h->thist[nb - 1])) return DMFE_ERR_INVALID;
    if (nb == 0 && t != 0.0) return DMFE_ERR_INVALID;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return fail(e, "hipSetDevice");
    const int L = h->L;
    YPoint* y = h->at<YPoint>(h->lo.rhs_y);
    YPoint* k = h->at<YPoint>(h->lo.rhs_k);
    HCHK(launch_interleave(L, yC, yR, y, h->stream));
    const dmfe_status st = eval_rhs(h, t, int(nb), y, k, nullptr);
    if (st != DMFE_OK) return st;
    HCHK(launch_deinterleave(L, k, outC, outR, h->stream));
    HCHK(hipMemcpyAsync(h->pinned, h->at<double>(h->lo.mue), 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HCHK(hipMemcpyAsync(h->pinned + 2, h->at<double>(h->lo.diag), 2 * sizeof(double), hipMemcpyDeviceToHost,
                        h->stream));
    HCHK(hipStreamSynchronize(h->stream));
    if (mu) *mu = h->pinned[0];
    if (diag) {
        diag[0] = h->pinned[2];
        diag[1] = h->pinned[3];
    }
    return DMFE_OK;
}

dmfe_status dmfe_read(dmfe_handle* h, int32_t field, int64_t first, int64_t count, void* dst, size_t dst_bytes,
                      int32_t dst_on_device, size_t* needed_bytes) {
    if (!h || first < 0 || count < 0) return DMFE_ERR_INVALID;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return fail(e, "hipSetDevice");
    const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    size_t need = 0;
    if (h->p.mode == DMFE_UNIFORM) {
        const int64_t rows = h->un + 1;
        switch (field) {
        case DMFE_F_C:
        case DMFE_F_R: {
            if (first + count > rows) return DMFE_ERR_INVALID;
            const size_t a = size_t(first) * (first + 1) / 2, b = size_t(first + count) * (first + count + 1) / 2;
            need = (b - a) * sizeof(double);
            if (needed_bytes) *needed_bytes = need;
            if (!dst) return DMFE_OK;
            if (dst_bytes < need) return DMFE_ERR_BUFFER;
            const double* src = h->at<double>(field == DMFE_F_C ? h->lo.uC : h->lo.uR) + a;
            HCHK(hipMemcpyAsync(dst, src, need, kind, h->stream));
            break;
        }
        case DMFE_F_ENERGY:
        case DMFE_F_T_GRID: {
            if (first + count > rows) return DMFE_ERR_INVALID;
            need = size_t(count) * sizeof(double);
            if (needed_bytes) *needed_bytes = need;
            if (!dst) return DMFE_OK;
            if (dst_bytes < need) return DMFE_ERR_BUFFER;
            if (field == DMFE_F_ENERGY) {
                HCHK(hipMemcpyAsync(dst, h->at<double>(h->lo.uE) + first, need, kind, h->stream));
            } else {
                std::vector<double> tg(count);
                for (int64_t q = 0; q < count; ++q) tg[q] = double(first + q) * h->p.h;
                HCHK(hipMemcpyAsync(dst, tg.data(), need, dst_on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost,
                                    h->stream));
                HCHK(hipStreamSynchronize(h->stream));
            }
            break;
        }
        default: return DMFE_ERR_INVALID;
        }
        HCHK(hipStreamSynchronize(h->stream));
        return DMFE_OK;
    }
    const int L = h->L;
    switch (field) {
    case DMFE_F_THETA:
    case DMFE_F_THETA_C:
    case DMFE_F_NU: {
        if (first + count > L) return DMFE_ERR_INVALID;
        need = size_t(count) * sizeof(double);
        if (needed_bytes) *needed_bytes = need;
        if (!dst) return DMFE_OK;
        if (dst_bytes < need) return DMFE_ERR_BUFFER;
        const size_t off = field == DMFE_F_THETA ? h->lo.th : field == DMFE_F_THETA_C ? h->lo.thc : h->lo.nu;
        HCHK(hipMemcpyAsync(dst, h->at<double>(off) + first, need, kind, h->stream));
        break;
    }
    case DMFE_F_T_GRID: {
        if (first + count > h->M) return DMFE_ERR_INVALID;
        need = size_t(count) * sizeof(double);
        if (needed_bytes) *needed_bytes = need;
        if (!dst) return DMFE_OK;
        if (dst_bytes < need) return DMFE_ERR_BUFFER;
        HCHK(hipMemcpyAsync(dst, h->at<double>(h->lo.thist) + first, need, kind, h->stream));
        break;
    }
    case DMFE_F_C:
    case DMFE_F_R:
    case DMFE_F_DC:
    case DMFE_F_DR: {
        if (first + count > h->M) return DMFE_ERR_INVALID;
        need = size_t(count) * L * sizeof(double);
        if (needed_bytes) *needed_bytes = need;
        if (!dst) return DMFE_OK;
        if (dst_bytes < need) return DMFE_ERR_BUFFER;
        const int fld = field - DMFE_F_C;
        double* io = h->at<double>(h->lo.io);
        for (int64_t n0 = 0; n0 < count; n0 += 64) {
            const int cnt = int(std::min<int64_t>(64, count - n0));
            HCHK(launch_pack_history(L, cnt, fld, h->at<int>(h->lo.slot) + first + n0, h->at<void>(h->lo.hist),
                                     h->fp32, io, h->stream));
            HCHK(hipMemcpyAsync(static_cast<char*>(dst) + size_t(n0) * L * sizeof(double), io,
                                size_t(cnt) * L * sizeof(double), kind, h->stream));
            HCHK(hipStreamSynchronize(h->stream));
        }
        break;
    }
    case DMFE_F_ENERGY:
    case DMFE_F_MU: {
        if (first + count > h->M) return DMFE_ERR_INVALID;
        need = size_t(count) * sizeof(double);
        if (needed_bytes) *needed_bytes = need;
        if (!dst) return DMFE_OK;
        if (dst_bytes < need) return DMFE_ERR_BUFFER;
        double* Eo = h->at<double>(h->lo.obs);
        double* Mo = Eo + h->Mc;
        HCHK(launch_slice_observables(h->m, L, h->at<double>(h->lo.nu), int(count), h->at<double>(h->lo.thist) + first,
                                      h->at<int>(h->lo.slot) + first, h->at<void>(h->lo.hist), h->fp32, Eo, Mo,
                                      h->stream));
        HCHK(hipMemcpyAsync(dst, field == DMFE_F_ENERGY ? Eo : Mo, need, kind, h->stream));
        break;
    }
    default: return DMFE_ERR_INVALID;
    }
    HCHK(hipStreamSynchronize(h->stream));
    return DMFE_OK;
}

dmfe_status dmfe_timing(dmfe_handle* h, int32_t enable) {
    if (!h) return DMFE_ERR_INVALID;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return fail(e, "hipSetDevice");
    HCHK(hipStreamSynchronize(h->stream));
    timing_drain(h);
    if (enable) {
        for (int k = 0; k < DMFE_K_COUNT; ++k) {
            h->kt_launches[k] = 0;
            h->kt_ms[k] = 0.0;
            h->kt_slices[k] = 0;
        }
    }
    h->timing = enable != 0;
    return DMFE_OK;
}

dmfe_status dmfe_timing_select(dmfe_handle* h, uint32_t mask) {
    if (!h || (mask >> DMFE_K_COUNT) != 0) return DMFE_ERR_INVALID;
    h->timing_mask = mask;
    return DMFE_OK;
}

dmfe_status dmfe_timing_read(dmfe_handle* h, int32_t kernel, int64_t* launches, double* total_ms,
                             int64_t* slices_read) {
    if (!h || kernel < 0 || kernel >= DMFE_K_COUNT) return DMFE_ERR_INVALID;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return fail(e, "hipSetDevice");
    HCHK(hipStreamSynchronize(h->stream));
    timing_drain(h);
    if (launches) *launches = h->kt_launches[kernel];
    if (total_ms) *total_ms = h->kt_ms[kernel];
    if (slices_read) *slices_read = h->kt_slices[kernel];
    return DMFE_OK;
}

}  // extern "C"
