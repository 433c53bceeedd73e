// Serving pool: many DMFE solves (a parameter sweep) stepped together.
//
// Requests are queued on submit and admitted when a slot is free and their
// device footprint fits in the pool's arena (first-fit over free ranges).
// Every tick advances each admitted solve by one RK stage: the stage
// combinations, the stage preps, the history integrals and the final
// combinations of all solves are each one batched launch (uneven L and M are
// handled per block through a per-launch instance table), followed by one
// synchronisation that returns the error norms of the solves that finished a
// step.  The controller then runs on the host per solve.  Finished solves keep
// their memory until released, so that results can be read.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "handle.h"

using namespace dmfe;
using namespace dmfe::core;

namespace {

double now_s() {
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

struct Request {
    uint64_t id;
    dmfe_params p;
    size_t bytes;
    double t_submit;
};

struct Instance {
    uint64_t id = 0;
    dmfe_handle* h = nullptr;
    size_t off = 0, bytes = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    bool done = false;
    dmfe_status status = DMFE_OK;
    int in_finish = 0;  // finishing its step in the current tick
};

}  // namespace

struct dmfe_pool {
    dmfe_pool_params pp{};
    int device = 0;
    hipStream_t stream = nullptr;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    std::map<size_t, size_t> free_ranges;  // offset -> size
    std::deque<Request> queue;
    std::vector<Instance> live;  // admitted, running or finished-unreleased
    std::vector<uint64_t> done_unpolled;
    uint64_t next_id = 1;
    int64_t ticks = 0;
    // batch descriptors: device buffers and pinned host staging
    char* d_desc = nullptr;
    char* h_desc = nullptr;  // descriptors filled per tick, laid out for max_instances
    char* h_pack = nullptr;  // the same, packed to the tick's counts for one short upload
    size_t desc_bytes = 0;
    double* d_eps = nullptr;
    double* h_eps = nullptr;

    size_t take(size_t bytes) {
        for (auto it = free_ranges.begin(); it != free_ranges.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, sz = it->second;
                free_ranges.erase(it);
                if (sz > bytes) free_ranges[off + bytes] = sz - bytes;
                return off;
            }
        }
        return size_t(-1);
    }
    void give(size_t off, size_t bytes) {
        auto it = free_ranges.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_ranges.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_ranges.erase(nx);
        }
        if (it != free_ranges.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_ranges.erase(it);
            }
        }
    }
    size_t bytes_free() const {
        size_t s = 0;
        for (auto& kv : free_ranges) s += kv.second;
        return s;
    }
    int running() const {
        int n = 0;
        for (auto& q : live) n += q.done ? 0 : 1;
        return n;
    }
};

namespace {

constexpr size_t kAlignDesc = 256;
inline size_t up256(size_t x) { return (x + kAlignDesc - 1) / kAlignDesc * kAlignDesc; }

// layout of one tick's descriptor block (capacity = max_instances)
struct DescLayout {
    size_t args, fb_hist, comb, fb_comb, prep, fin, total;
};
DescLayout desc_layout(int cap) {
    DescLayout d{};
    size_t o = 0;
    d.args = o;
    o += up256(sizeof(StageArgs) * cap);
    d.fb_hist = o;
    o += up256(sizeof(int) * (cap + 1));
    d.comb = o;
    o += up256(sizeof(CombineDesc) * cap);
    d.fb_comb = o;
    o += up256(sizeof(int) * (cap + 1));
    d.prep = o;
    o += up256(sizeof(PrepDesc) * cap);
    d.fin = o;
    o += up256(sizeof(FinishDesc) * cap);
    d.total = o;
    return d;
}

dmfe_status admit(dmfe_pool* P) {
    while (!P->queue.empty() && int(P->live.size()) < P->pp.max_instances) {
        Request& r = P->queue.front();
        const size_t off = P->take(r.bytes);
        if (off == size_t(-1)) break;  // wait for memory
        dmfe_resources res{};
        res.device = P->device;
        res.stream = P->stream;
        res.workspace = P->arena + off;
        res.workspace_bytes = r.bytes;
        dmfe_handle* h = nullptr;
        const dmfe_status st = dmfe_create(&r.p, &res, &h);
        Instance q;
        q.id = r.id;
        q.off = off;
        q.bytes = r.bytes;
        q.t_submit = r.t_submit;
        q.t_admit = now_s();
        if (st != DMFE_OK) {
            P->give(off, r.bytes);
            q.done = true;
            q.status = st;
            q.t_done = q.t_admit;
            P->done_unpolled.push_back(q.id);
            P->queue.pop_front();
            continue;  // a request that cannot be created is reported, not retried
        }
        q.h = h;
        P->live.push_back(q);
        P->queue.pop_front();
    }
    return DMFE_OK;
}

void finish_instance(dmfe_pool* P, Instance& q, dmfe_status st) {
    q.done = true;
    q.status = st;
    q.t_done = now_s();
    P->done_unpolled.push_back(q.id);
}

// One tick: every running solve advances by one RK stage.
dmfe_status tick(dmfe_pool* P) {
    admit(P);
    const DescLayout dl = desc_layout(P->pp.max_instances);
    StageArgs* a_args = reinterpret_cast<StageArgs*>(P->h_desc + dl.args);
    int* a_fbh = reinterpret_cast<int*>(P->h_desc + dl.fb_hist);
    CombineDesc* a_comb = reinterpret_cast<CombineDesc*>(P->h_desc + dl.comb);
    int* a_fbc = reinterpret_cast<int*>(P->h_desc + dl.fb_comb);
    PrepDesc* a_prep = reinterpret_cast<PrepDesc*>(P->h_desc + dl.prep);
    FinishDesc* a_fin = reinterpret_cast<FinishDesc*>(P->h_desc + dl.fin);
    int n_eval = 0, n_comb = 0, n_fin = 0, hist_blocks = 0, comb_blocks = 0, nb_max = 0, pmax = 2, fp32 = -1;
    std::vector<int> fin_of;  // live index of each finishing solve
    for (size_t qi = 0; qi < P->live.size(); ++qi) {
        Instance& q = P->live[qi];
        q.in_finish = 0;
        if (q.done) continue;
        dmfe_handle* h = q.h;
        if (!h->cur.active) {
            if (h->t >= h->p.t_max) {
                finish_instance(P, q, DMFE_DONE);
                continue;
            }
            const dmfe_status st = step_begin(h);
            if (st != DMFE_OK) {
                finish_instance(P, q, st);
                continue;
            }
        }
        auto& c = h->cur;
        const Tableau& T = *c.T;
        // first-same-as-last: k_0 already holds the last step's final stage (written on accept),
        // so the step's first stage needs no work and its second runs in this tick
        if (c.st == 0 && h->fsal_valid) c.st = 1;
        const int L = h->L, st = c.st;
        YPoint* y0 = h->at<YPoint>(h->lo.y);
        YPoint* ys = h->at<YPoint>(h->lo.ys);
        YPoint* kb = h->at<YPoint>(h->lo.k);
        YPoint* kst = kb + size_t(st) * L;
        const double tst = c.tn + T.c[st] * c.dt;
        if (fp32 < 0) fp32 = h->fp32;
        const YPoint* ycur = y0;
        int nb = c.M - 1;
        void* store = slot_ptr(h, h->slot[c.M - 1]);
        if (st > 0) {
            CombineDesc& cd = a_comb[n_comb];
            cd.y0 = y0;
            cd.k = kb;
            cd.ys = ys;
            cd.L = L;
            cd.nk = st;
            cd.dt = c.dt;
            for (int l = 0; l < 10; ++l) cd.a[l] = l < st ? T.A[st][l] : 0.0;
            a_fbc[n_comb] = comb_blocks;
            comb_blocks += (L + kCombineBlock - 1) / kCombineBlock;
            ++n_comb;
            ycur = ys;
            nb = c.M;
            store = (T.fsal && st == T.S - 1) ? slot_ptr(h, c.next_slot) : nullptr;
        }
        PrepDesc& pd = a_prep[n_eval];
        pd.y = ycur;
        pd.nu = h->at<double>(h->lo.nu);
        pd.mue = h->at<double>(h->lo.mue);
        pd.stage = stage_slot(h);
        pd.L = L;
        pd.fp32 = h->fp32;
        pd.t = tst;
        pd.m = h->m;
        a_args[n_eval] = stage_args(h, tst, nb, ycur, kst, store);
        a_fbh[n_eval] = hist_blocks;
        hist_blocks += (L + hist_rows_per_block(h->fp32) - 1) / hist_rows_per_block(h->fp32);
        nb_max = std::max(nb_max, nb);
        pmax = std::max(pmax, h->m.pmax);
        ++n_eval;
        h->rhs_evals += 1;
        c.st = st + 1;
        if (c.st == T.S) {
            FinishDesc& fd = a_fin[n_fin];
            fd.y0 = y0;
            fd.k = kb;
            fd.ynew = h->at<YPoint>(h->lo.ynew);
            fd.eps = P->d_eps + n_fin;
            fd.L = L;
            fd.nk = T.S;
            fd.dt = c.dt;
            for (int l = 0; l < 10; ++l) {
                fd.b[l] = l < T.S ? T.b[l] : 0.0;
                fd.e[l] = l < T.S ? T.e[l] : 0.0;
            }
            q.in_finish = 1;
            fin_of.push_back(int(qi));
            ++n_fin;
        }
    }
    a_fbh[n_eval] = hist_blocks;
    a_fbc[n_comb] = comb_blocks;
    if (n_eval + n_comb + n_fin > 0) {
        // upload only this tick's entries: the sections packed to their counts
        DescLayout pl{};
        size_t o = 0;
        pl.args = o;
        o += up256(sizeof(StageArgs) * n_eval);
        pl.fb_hist = o;
        o += up256(sizeof(int) * (n_eval + 1));
        pl.comb = o;
        o += up256(sizeof(CombineDesc) * n_comb);
        pl.fb_comb = o;
        o += up256(sizeof(int) * (n_comb + 1));
        pl.prep = o;
        o += up256(sizeof(PrepDesc) * n_eval);
        pl.fin = o;
        o += up256(sizeof(FinishDesc) * n_fin);
        pl.total = o;
        std::memcpy(P->h_pack + pl.args, P->h_desc + dl.args, sizeof(StageArgs) * n_eval);
        std::memcpy(P->h_pack + pl.fb_hist, P->h_desc + dl.fb_hist, sizeof(int) * (n_eval + 1));
        std::memcpy(P->h_pack + pl.comb, P->h_desc + dl.comb, sizeof(CombineDesc) * n_comb);
        std::memcpy(P->h_pack + pl.fb_comb, P->h_desc + dl.fb_comb, sizeof(int) * (n_comb + 1));
        std::memcpy(P->h_pack + pl.prep, P->h_desc + dl.prep, sizeof(PrepDesc) * n_eval);
        std::memcpy(P->h_pack + pl.fin, P->h_desc + dl.fin, sizeof(FinishDesc) * n_fin);
        // the previous tick ended with a stream synchronisation, so h_pack is free to refill
        HCHK(hipMemcpyAsync(P->d_desc, P->h_pack, pl.total, hipMemcpyHostToDevice, P->stream));
        const char* D = P->d_desc;
        HCHK(launch_rk_combine_multi(reinterpret_cast<const CombineDesc*>(D + pl.comb),
                                     reinterpret_cast<const int*>(D + pl.fb_comb), n_comb, comb_blocks, P->stream));
        HCHK(launch_stage_prep_multi(reinterpret_cast<const PrepDesc*>(D + pl.prep), n_eval, pmax, P->stream));
        HCHK(launch_hist_integral_multi(reinterpret_cast<const StageArgs*>(D + pl.args),
                                        reinterpret_cast<const int*>(D + pl.fb_hist), n_eval, hist_blocks, 10, pmax,
                                        fp32 < 0 ? 0 : fp32, nb_max, P->stream));
        HCHK(launch_rk_finish_multi(reinterpret_cast<const FinishDesc*>(D + pl.fin), n_fin, P->stream));
        if (n_fin > 0)
            HCHK(hipMemcpyAsync(P->h_eps, P->d_eps, sizeof(double) * n_fin, hipMemcpyDeviceToHost, P->stream));
        HCHK(hipStreamSynchronize(P->stream));
    }
    for (int f = 0; f < n_fin; ++f) {
        Instance& q = P->live[fin_of[f]];
        const dmfe_status st = step_decide(q.h, P->h_eps[f]);
        if (st != DMFE_OK) finish_instance(P, q, st);
        else if (q.h->t >= q.h->p.t_max) finish_instance(P, q, DMFE_DONE);
    }
    P->ticks += 1;
    return DMFE_OK;
}

Instance* find_live(dmfe_pool* P, uint64_t id) {
    for (auto& q : P->live)
        if (q.id == id) return &q;
    return nullptr;
}

}  // namespace

extern "C" {

dmfe_status dmfe_pool_create(const dmfe_pool_params* pp, const dmfe_resources* res, dmfe_pool** out) {
    if (!pp || !out || pp->max_instances < 1 || pp->max_instances > 4096) return DMFE_ERR_INVALID;
    *out = nullptr;
    dmfe_pool* P = new (std::nothrow) dmfe_pool();
    if (!P) return DMFE_ERR_NOMEM;
    P->pp = *pp;
    P->device = res ? res->device : 0;
    P->stream = res ? reinterpret_cast<hipStream_t>(res->stream) : nullptr;
    hipError_t e = hipSetDevice(P->device);
    if (e != hipSuccess) {
        delete P;
        return fail(e, "hipSetDevice");
    }
    if (res && res->workspace) {
        P->arena = static_cast<char*>(res->workspace);
        P->arena_bytes = pp->max_bytes ? std::min(pp->max_bytes, res->workspace_bytes) : res->workspace_bytes;
    } else {
        delete P;
        return DMFE_ERR_INVALID;  // the arena is caller-owned device memory
    }
    P->free_ranges[0] = P->arena_bytes;
    const DescLayout dl = desc_layout(pp->max_instances);
    P->desc_bytes = dl.total;
    if (hipMalloc(reinterpret_cast<void**>(&P->d_desc), dl.total) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&P->h_desc), dl.total, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&P->h_pack), dl.total, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&P->d_eps), sizeof(double) * pp->max_instances) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&P->h_eps), sizeof(double) * pp->max_instances,
                      hipHostMallocDefault) != hipSuccess) {
        dmfe_pool_destroy(P);
        return DMFE_ERR_NOMEM;
    }
    std::memset(P->h_desc, 0, dl.total);
    *out = P;
    return DMFE_OK;
}

dmfe_status dmfe_pool_submit(dmfe_pool* P, const dmfe_params* p, uint64_t* id) {
    if (!P || !p || !id) return DMFE_ERR_INVALID;
    if (p->mode != DMFE_ADAPTIVE) return DMFE_ERR_INVALID;
    size_t bytes = 0;
    const dmfe_status st = dmfe_footprint(p, &bytes);
    if (st != DMFE_OK) return st;
    // the batched kernel serves the default stencil
    if ((p->s != 0 && p->s != 10) || p->theta_interp != DMFE_INTERP_INDEX_LAGRANGE || p->log_r != 0 ||
        (p->M_cap == 0 ? p->L : p->M_cap) > 16384)
        return DMFE_ERR_UNSUPPORTED;
    if (bytes > P->arena_bytes) return DMFE_ERR_NOMEM;
    // one pool serves one history precision (the batched kernel is instantiated per precision)
    for (auto& q : P->live)
        if (!q.done && q.h && q.h->p.precision != p->precision) return DMFE_ERR_UNSUPPORTED;
    for (auto& r : P->queue)
        if (r.p.precision != p->precision) return DMFE_ERR_UNSUPPORTED;
    Request r;
    r.id = P->next_id++;
    r.p = *p;
    r.bytes = (bytes + 255) / 256 * 256;
    r.t_submit = now_s();
    P->queue.push_back(r);
    *id = r.id;
    return DMFE_OK;
}

dmfe_status dmfe_pool_run(dmfe_pool* P, int64_t max_ticks, dmfe_pool_stats* stats) {
    if (!P || max_ticks < 0) return DMFE_ERR_INVALID;
    hipError_t e = hipSetDevice(P->device);
    if (e != hipSuccess) return fail(e, "hipSetDevice");
    for (int64_t k = 0; k < max_ticks; ++k) {
        admit(P);
        if (P->running() == 0) break;
        const dmfe_status st = tick(P);
        if (st != DMFE_OK) return st;
    }
    admit(P);
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->running = P->running();
        stats->queued = int32_t(P->queue.size());
        stats->finished_unreleased = int32_t(P->live.size()) - stats->running;
        stats->ticks = P->ticks;
        stats->bytes_free = P->bytes_free();
        stats->bytes_total = P->arena_bytes;
    }
    return DMFE_OK;
}

dmfe_status dmfe_pool_poll(dmfe_pool* P, uint64_t* done_ids, int32_t cap, int32_t* n_done) {
    if (!P || !n_done || cap < 0) return DMFE_ERR_INVALID;
    const int n = std::min<int>(cap, int(P->done_unpolled.size()));
    for (int q = 0; q < n; ++q) done_ids[q] = P->done_unpolled[q];
    P->done_unpolled.erase(P->done_unpolled.begin(), P->done_unpolled.begin() + n);
    *n_done = n;
    return DMFE_OK;
}

dmfe_status dmfe_pool_result(dmfe_pool* P, uint64_t id, dmfe_step_info* info, dmfe_pool_times* times) {
    if (!P) return DMFE_ERR_INVALID;
    Instance* q = find_live(P, id);
    if (!q) return DMFE_ERR_INVALID;
    if (info) {
        if (q->h) fill_info(q->h, info);
        else std::memset(info, 0, sizeof(*info));
    }
    if (times) {
        times->status = q->done ? q->status : DMFE_OK;
        times->done = q->done ? 1 : 0;
        times->queue_s = q->t_admit - q->t_submit;
        times->service_s = (q->done ? q->t_done : now_s()) - q->t_admit;
        times->total_s = (q->done ? q->t_done : now_s()) - q->t_submit;
    }
    return DMFE_OK;
}

dmfe_status dmfe_pool_read(dmfe_pool* P, uint64_t id, int32_t field, int64_t first, int64_t count, void* dst,
                           size_t dst_bytes, int32_t dst_on_device, size_t* needed_bytes) {
    if (!P) return DMFE_ERR_INVALID;
    Instance* q = find_live(P, id);
    if (!q || !q->h) return DMFE_ERR_INVALID;
    return dmfe_read(q->h, field, first, count, dst, dst_bytes, dst_on_device, needed_bytes);
}

dmfe_status dmfe_pool_set_history(dmfe_pool* P, uint64_t id, int64_t M, int64_t nb, const double* t_hist,
                                  const double* C, const double* R, const double* dC, const double* dR,
                                  int32_t src_on_device, double dt, int32_t scheme) {
    if (!P) return DMFE_ERR_INVALID;
    Instance* q = find_live(P, id);
    // admitted, still running, and between two steps (no stage of it in flight)
    if (!q || !q->h || q->done || q->h->cur.active) return DMFE_ERR_INVALID;
    return dmfe_set_history(q->h, M, nb, t_hist, C, R, dC, dR, src_on_device, dt, scheme);
}

dmfe_status dmfe_pool_release(dmfe_pool* P, uint64_t id) {
    if (!P) return DMFE_ERR_INVALID;
    for (size_t k = 0; k < P->live.size(); ++k) {
        Instance& q = P->live[k];
        if (q.id != id) continue;
        if (!q.done) return DMFE_ERR_INVALID;  // still running
        if (q.h) dmfe_destroy(q.h);
        P->give(q.off, q.bytes);
        P->live.erase(P->live.begin() + long(k));
        return DMFE_OK;
    }
    return DMFE_ERR_INVALID;
}

void dmfe_pool_destroy(dmfe_pool* P) {
    if (!P) return;
    (void)hipSetDevice(P->device);
    if (P->stream) (void)hipStreamSynchronize(P->stream);
    for (auto& q : P->live)
        if (q.h) dmfe_destroy(q.h);
    if (P->d_desc) (void)hipFree(P->d_desc);
    if (P->h_desc) (void)hipHostFree(P->h_desc);
    if (P->h_pack) (void)hipHostFree(P->h_pack);
    if (P->d_eps) (void)hipFree(P->d_eps);
    if (P->h_eps) (void)hipHostFree(P->h_eps);
    delete P;
}

}  // extern "C"
