// Internal: the solver handle and the core routines shared by the C-ABI
// (api.hip) and the serving pool (pool.hip).  Not part of the C-ABI.
#pragma once

#include <string>
#include <vector>

#include "dmfe_internal.h"

namespace dmfe {
namespace core {

// Butcher tableau of up to 10 stages with the embedded error weights e = b - bhat.
struct Tableau {
    int S = 0;
    double A[10][10] = {};
    double b[10] = {};
    double e[10] = {};
    double c[10] = {};
    bool fsal = false;  // last stage is evaluated at y_new (c = 1, last row of A = b)
};

struct Layout {
    size_t hist, lhist, thist, slot, th, thc, nu, bw, X, Xd, y, ys, ynew, k, mue, eps, diag, eps_n, eps_part, obs, rhs_y,
        rhs_k, io, total;
    // uniform
    size_t uC, uR, uE, uy0, uy1, uys, uk;
};

// Real-axis stability limits of the two RK schemes (|R(-x)| <= 1 on [0, limit]),
// truncated: Dormand-Prince 5 and SSPRK(10,4).
constexpr double kDp5Limit = 3.3065;
constexpr double kSspLimit = 13.917;

struct CkptWriter;  // background checkpoint writer (checkpoint.hip)

}  // namespace core
}  // namespace dmfe

struct dmfe_handle {
    dmfe_params p{};
    dmfe::core::Layout lo{};
    int device = 0;
    hipStream_t stream = nullptr;
    char* base = nullptr;
    bool owns = false;
    dmfe::Model m{};
    // adaptive
    int L = 0, s = 10, Mc = 0;
    int fp32 = 0;  // history stored as HPoint32
    double gamma = 0, Dg = 0, xscale = 0, eg = 0, egi = 0;
    std::vector<double> th, thc, nu;
    double fh_c[16] = {};  // index Floater-Hormann coefficients (every stencil base alike)
    std::vector<double> thist;  // logical order
    std::vector<int> slot;      // logical order
    std::vector<int> free_slots;
    int M = 0, nb_valid = 0;
    double t = 0, dt = 0, eps_rk = 0;
    int scheme = DMFE_SCHEME_DP5;
    bool fsal_valid = false;
    dmfe::core::Tableau dp5, ssp;
    double* pinned = nullptr;  // host staging for small readbacks
    // uniform
    int64_t un = 0;  // rows stored - 1
    int ucur = 0;    // which of uy0/uy1 holds the current row
    // counters
    int64_t accepted = 0, rejected = 0, reverts = 0, n_sparsify = 0, removed = 0, rhs_evals = 0;
    // per-kernel timing (HIP events on the handle's stream)
    struct EvPair {
        hipEvent_t a = nullptr, b = nullptr;
        int kernel = 0;
        int64_t slices = 0;
    };
    bool timing = false;
    uint32_t timing_mask = (1u << DMFE_K_COUNT) - 1;  // kernels timed when timing is on
    int64_t kt_launches[DMFE_K_COUNT] = {};
    double kt_ms[DMFE_K_COUNT] = {};
    int64_t kt_slices[DMFE_K_COUNT] = {};
    std::vector<EvPair> ev_pool, ev_pending;

    // the step in flight (stage-by-stage driving, used by dmfe_step and the serving pool)
    struct StepCtx {
        int active = 0;
        int st = 0;                   // next stage to evaluate
        const dmfe::core::Tableau* T = nullptr;
        int M = 0;                    // slices at the start of the step
        double dt = 0.0, tn = 0.0;
        int next_slot = -1;
    } cur;

    dmfe::core::CkptWriter* ckpt = nullptr;  // at most one checkpoint write in flight

    template <class T> T* at(size_t off) const { return reinterpret_cast<T*>(base + off); }
};


namespace dmfe {
namespace core {

void set_error(const std::string& msg);
const char* last_error();
dmfe_status fail(hipError_t e, const char* what);
dmfe_status fail_msg(dmfe_status s, const std::string& msg);  // records msg, returns s
dmfe_status ckpt_join(dmfe_handle* h);   // waits for the handle's checkpoint write, returns its status
void ckpt_release(dmfe_handle* h);       // waits for it and frees the writer
#define HCHK(expr)                                            \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) return ::dmfe::core::fail(e_, #expr); \
    } while (0)

Tableau make_dp5();
Tableau make_ssprk104();
Layout make_layout(const dmfe_params& p);
dmfe_status validate(const dmfe_params* p);
Model make_model(const dmfe_params& p);
double f2_at_one(const Model& m);

dmfe_handle::EvPair* timing_begin(dmfe_handle* h, int kernel, int64_t slices);
void timing_end(dmfe_handle* h, dmfe_handle::EvPair* p);
void timing_drain(dmfe_handle* h);

// Per-evaluation buffers of one right-hand side: the stage slice in history format
// and its log mirror (log-R option), mu(t) and E(t), the computed diagonal values.
struct StageBufs {
    void* stage;
    LogPoint* lstage;
    double* mue;
    double* diag;
};
StageBufs handle_bufs(const dmfe_handle* h);  // the handle's own, in its workspace
StageArgs stage_args(const dmfe_handle* h, double t, int nb, const YPoint* y, YPoint* kout, void* store,
                     const StageBufs& b);
StageArgs stage_args(const dmfe_handle* h, double t, int nb, const YPoint* y, YPoint* kout, void* store);
void* stage_slot(const dmfe_handle* h);  // the stage slice in history format, after the Mc slots
LogPoint* log_mirror(const dmfe_handle* h);  // log-R option: mirror of the Mc slots and the stage slot, else null
dmfe_status rebuild_log_mirror(dmfe_handle* h);  // mirror of the M stored slices from their stored values
// one right-hand side into b's buffers; `timed` records the launches for dmfe_timing
dmfe_status eval_rhs(dmfe_handle* h, double t, int nb, const YPoint* y, YPoint* kout, void* store,
                     const StageBufs& b, bool timed);
dmfe_status eval_rhs(dmfe_handle* h, double t, int nb, const YPoint* y, YPoint* kout, void* store);
size_t point_bytes(const dmfe_handle* h);
void* slot_ptr(dmfe_handle* h, int slot);
dmfe_status upload_order(dmfe_handle* h);
dmfe_status sparsify_pass(dmfe_handle* h, int64_t* removed_out);
void fill_info(const dmfe_handle* h, dmfe_step_info* info);

// Stage-by-stage driving of one adaptive step:
//   step_begin   runs automatic sparsification if the history is full and
//                fixes the scheme, dt and the slot of the next slice;
//   step_stage   enqueues the next stage (combination + right-hand side);
//   step_finish  enqueues the final combination and the error norm, whose
//                value is copied to h->pinned[0];
//   step_decide  applies the controller to that value (after the stream has
//                been synchronised) and enqueues append or revert.
dmfe_status step_begin(dmfe_handle* h);
dmfe_status step_stage(dmfe_handle* h);
dmfe_status step_finish(dmfe_handle* h);
dmfe_status step_decide(dmfe_handle* h, double err);

}  // namespace core
}  // namespace dmfe
