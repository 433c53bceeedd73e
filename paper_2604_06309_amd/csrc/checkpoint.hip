// Checkpoint and resume of an adaptive solve: the solver state is written to
// a binary file and a new handle restored from it continues bitwise as the
// original would have.  A save copies the device state to host memory before
// it returns; the file itself is written synchronously or by one background
// thread per handle (a second save waits for the first).
//
// File format (version 2, host byte order):
//   CkptHeader
//   t_n of the M stored slices               M doubles, logical order
//   the state y(t)                           L YPoint (FP64; an FP32 history holds only its rounding)
//   F(t, y) kept for reuse by DP5's first     L YPoint (zeros when none is kept)
//   stage
//   the M stored slices                      M x L points in the handle's storage format, logical order
// The header records the solve's parameters, the controller state and the
// counters, and an FNV-1a checksum (64-bit words) over the header, with its
// checksum field zeroed, followed by the payload: an altered parameter, state
// or counter is refused like an altered history.
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "handle.h"

namespace dmfe {
namespace core {

namespace {

constexpr char kMagic[8] = {'D', 'M', 'F', 'E', 'C', 'K', 'P', '1'};
constexpr uint32_t kVersion = 2;

struct CkptHeader {
    char magic[8];
    uint32_t version;
    uint32_t header_bytes;
    dmfe_params params;
    int64_t M, nb_valid;
    int64_t accepted, rejected, reverts, n_sparsify, removed, rhs_evals;
    double t, dt, eps_rk;
    int32_t scheme, fsal_valid, point_bytes, L;
    uint64_t payload_bytes;
    uint64_t checksum;
};

constexpr uint64_t kFnvBasis = 1469598103934665603ull;
uint64_t fnv1a64(const unsigned char* p, size_t n, uint64_t h = kFnvBasis) {
    size_t q = 0;
    for (; q + 8 <= n; q += 8) {
        uint64_t w;
        std::memcpy(&w, p + q, 8);
        h = (h ^ w) * 1099511628211ull;
    }
    for (; q < n; ++q) h = (h ^ p[q]) * 1099511628211ull;
    return h;
}

// Checksum of the header bytes as written (checksum field taken as zero) and
// the payload.  The header is hashed from a byte copy, so padding bytes count
// exactly as they are stored.
uint64_t file_checksum(const unsigned char (&hb)[sizeof(CkptHeader)], const std::vector<unsigned char>& payload) {
    unsigned char z[sizeof(CkptHeader)];
    std::memcpy(z, hb, sizeof(z));
    std::memset(z + offsetof(CkptHeader, checksum), 0, sizeof(uint64_t));
    return fnv1a64(payload.data(), payload.size(), fnv1a64(z, sizeof(z)));
}

dmfe_status write_file(const std::string& path, const CkptHeader& hdr, const std::vector<unsigned char>& payload) {
    unsigned char hb[sizeof(CkptHeader)];
    std::memcpy(hb, &hdr, sizeof(hb));
    const uint64_t sum = file_checksum(hb, payload);
    std::memcpy(hb + offsetof(CkptHeader, checksum), &sum, sizeof(sum));
    FILE* f = std::fopen(path.c_str(), "wb");
    if (!f) return fail_msg(DMFE_ERR_INVALID, "checkpoint: cannot open " + path + " for writing");
    const bool ok = std::fwrite(hb, sizeof(hb), 1, f) == 1 &&
                    std::fwrite(payload.data(), 1, payload.size(), f) == payload.size() && std::fflush(f) == 0;
    const bool closed = std::fclose(f) == 0;
    if (!ok || !closed) return fail_msg(DMFE_ERR_INVALID, "checkpoint: write to " + path + " failed");
    return DMFE_OK;
}

}  // namespace

struct CkptWriter {
    std::thread th;
    dmfe_status status = DMFE_OK;
};

dmfe_status ckpt_join(dmfe_handle* h) {
    if (!h->ckpt) return DMFE_OK;
    if (h->ckpt->th.joinable()) h->ckpt->th.join();
    return h->ckpt->status;
}

void ckpt_release(dmfe_handle* h) {
    (void)ckpt_join(h);
    delete h->ckpt;
    h->ckpt = nullptr;
}

}  // namespace core
}  // namespace dmfe

using namespace dmfe;
using namespace dmfe::core;

extern "C" {

dmfe_status dmfe_checkpoint_save(dmfe_handle* h, const char* path, int32_t async) {
    if (!h || !path || h->p.mode != DMFE_ADAPTIVE) return h && path ? DMFE_ERR_UNSUPPORTED : DMFE_ERR_INVALID;
    if (h->cur.active) return fail_msg(DMFE_ERR_INVALID, "checkpoint: a step is in flight");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return fail(e, "hipSetDevice");
    // at most one write in flight: finish the previous one first
    const dmfe_status prev = ckpt_join(h);
    if (prev != DMFE_OK) return prev;
    const int L = h->L, M = h->M;
    const size_t pb = point_bytes(h);
    const size_t yb = sizeof(YPoint) * size_t(L);
    std::vector<unsigned char> payload(sizeof(double) * M + 2 * yb + size_t(M) * L * pb);
    unsigned char* q = payload.data();
    std::memcpy(q, h->thist.data(), sizeof(double) * M);
    q += sizeof(double) * M;
    HCHK(hipStreamSynchronize(h->stream));
    HCHK(hipMemcpyAsync(q, h->at<YPoint>(h->lo.y), yb, hipMemcpyDeviceToHost, h->stream));
    q += yb;
    if (h->fsal_valid)
        HCHK(hipMemcpyAsync(q, h->at<YPoint>(h->lo.k) + size_t(6) * L, yb, hipMemcpyDeviceToHost, h->stream));
    q += yb;
    for (int n = 0; n < M; ++n) {
        HCHK(hipMemcpyAsync(q, slot_ptr(h, h->slot[n]), size_t(L) * pb, hipMemcpyDeviceToHost, h->stream));
        q += size_t(L) * pb;
    }
    HCHK(hipStreamSynchronize(h->stream));
    CkptHeader hdr{};
    std::memcpy(hdr.magic, kMagic, 8);
    hdr.version = kVersion;
    hdr.header_bytes = sizeof(CkptHeader);
    hdr.params = h->p;
    hdr.M = M;
    hdr.nb_valid = h->nb_valid;
    hdr.accepted = h->accepted;
    hdr.rejected = h->rejected;
    hdr.reverts = h->reverts;
    hdr.n_sparsify = h->n_sparsify;
    hdr.removed = h->removed;
    hdr.rhs_evals = h->rhs_evals;
    hdr.t = h->t;
    hdr.dt = h->dt;
    hdr.eps_rk = h->eps_rk;
    hdr.scheme = h->scheme;
    hdr.fsal_valid = h->fsal_valid ? 1 : 0;
    hdr.point_bytes = int32_t(pb);
    hdr.L = L;
    hdr.payload_bytes = payload.size();
    if (!async) return write_file(path, hdr, payload);
    if (!h->ckpt) h->ckpt = new CkptWriter;
    h->ckpt->status = DMFE_OK;
    CkptWriter* w = h->ckpt;
    w->th = std::thread([w, p = std::string(path), hdr, buf = std::move(payload)]() {
        w->status = write_file(p, hdr, buf);
    });
    return DMFE_OK;
}

dmfe_status dmfe_checkpoint_wait(dmfe_handle* h) {
    if (!h) return DMFE_ERR_INVALID;
    return ckpt_join(h);
}

dmfe_status dmfe_checkpoint_load(const char* path, const dmfe_resources* res, dmfe_handle** out) {
    if (!path || !out) return DMFE_ERR_INVALID;
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail_msg(DMFE_ERR_INVALID, std::string("checkpoint: cannot open ") + path);
    CkptHeader hdr{};
    unsigned char hb[sizeof(CkptHeader)];
    const bool got = std::fread(hb, sizeof(hb), 1, f) == 1;
    if (got) std::memcpy(&hdr, hb, sizeof(hb));
    const bool hdr_ok = got && std::memcmp(hdr.magic, kMagic, 8) == 0 && hdr.version == kVersion &&
                        hdr.header_bytes == sizeof(CkptHeader);
    if (!hdr_ok) {
        std::fclose(f);
        return fail_msg(DMFE_ERR_INVALID, std::string("checkpoint: not a version-2 checkpoint: ") + path);
    }
    const dmfe_params& p = hdr.params;
    const size_t pb = p.precision == DMFE_FP32_COMP ? sizeof(HPoint32) : sizeof(HPoint);
    const int Mc = p.M_cap > 0 ? p.M_cap : p.L;
    const bool shape_ok = p.mode == DMFE_ADAPTIVE && hdr.L == p.L && hdr.point_bytes == int32_t(pb) && hdr.M >= 1 &&
                          hdr.M <= Mc && hdr.nb_valid >= hdr.M - 1 && hdr.nb_valid <= hdr.M &&
                          hdr.payload_bytes == sizeof(double) * hdr.M + 2 * sizeof(YPoint) * size_t(p.L) +
                                                   size_t(hdr.M) * p.L * pb;
    if (!shape_ok) {
        std::fclose(f);
        return fail_msg(DMFE_ERR_INVALID, std::string("checkpoint: inconsistent header: ") + path);
    }
    std::vector<unsigned char> payload(hdr.payload_bytes);
    const bool read_ok = std::fread(payload.data(), 1, payload.size(), f) == payload.size();
    std::fclose(f);
    if (!read_ok || file_checksum(hb, payload) != hdr.checksum)
        return fail_msg(DMFE_ERR_INVALID, std::string("checkpoint: truncated or corrupted: ") + path);

    dmfe_handle* h = nullptr;
    dmfe_status st = dmfe_create(&p, res, &h);
    if (st != DMFE_OK) return st;
    auto bail = [&](dmfe_status s) {
        dmfe_destroy(h);
        return s;
    };
    const int L = h->L, M = int(hdr.M);
    const size_t yb = sizeof(YPoint) * size_t(L);
    const unsigned char* q = payload.data();
    h->thist.assign(reinterpret_cast<const double*>(q), reinterpret_cast<const double*>(q) + M);
    q += sizeof(double) * M;
    h->slot.resize(M);
    for (int n = 0; n < M; ++n) h->slot[n] = n;
    h->free_slots.clear();
    for (int s = h->Mc - 1; s >= M; --s) h->free_slots.push_back(s);
    h->M = M;
    h->nb_valid = int(hdr.nb_valid);
    h->t = hdr.t;
    h->dt = hdr.dt;
    h->eps_rk = hdr.eps_rk;
    h->scheme = hdr.scheme;
    h->fsal_valid = hdr.fsal_valid != 0;
    h->accepted = hdr.accepted;
    h->rejected = hdr.rejected;
    h->reverts = hdr.reverts;
    h->n_sparsify = hdr.n_sparsify;
    h->removed = hdr.removed;
    h->rhs_evals = hdr.rhs_evals;
    hipError_t e = hipSuccess;
    if ((e = hipMemcpyAsync(h->at<YPoint>(h->lo.y), q, yb, hipMemcpyHostToDevice, h->stream)) != hipSuccess)
        return bail(fail(e, "hipMemcpyAsync"));
    q += yb;
    if ((e = hipMemcpyAsync(h->at<YPoint>(h->lo.k) + size_t(6) * L, q, yb, hipMemcpyHostToDevice, h->stream)) !=
        hipSuccess)
        return bail(fail(e, "hipMemcpyAsync"));
    // the next step's first stage reads it from k_0 (first-same-as-last)
    if (h->fsal_valid &&
        (e = hipMemcpyAsync(h->at<YPoint>(h->lo.k), q, yb, hipMemcpyHostToDevice, h->stream)) != hipSuccess)
        return bail(fail(e, "hipMemcpyAsync"));
    q += yb;
    // slots 0..M-1 are contiguous at the start of the history
    if ((e = hipMemcpyAsync(slot_ptr(h, 0), q, size_t(M) * L * pb, hipMemcpyHostToDevice, h->stream)) != hipSuccess)
        return bail(fail(e, "hipMemcpyAsync"));
    st = upload_order(h);  // also finishes the copies above before the payload goes away
    if (st == DMFE_OK) st = rebuild_log_mirror(h);  // log-R option: a function of the stored values
    if (st != DMFE_OK) return bail(st);
    *out = h;
    return DMFE_OK;
}

dmfe_status dmfe_snapshot_save(dmfe_handle* h, const char* path, int32_t theta_stride, int32_t slice_stride) {
    if (!h || !path || theta_stride < 1 || slice_stride < 1) return DMFE_ERR_INVALID;
    if (h->p.mode != DMFE_ADAPTIVE) return DMFE_ERR_UNSUPPORTED;
    if (h->cur.active) return fail_msg(DMFE_ERR_INVALID, "snapshot: a step is in flight");
    const int L = h->L, M = h->M;
    std::vector<int64_t> nodes, slices;
    for (int i = 0; i < L; i += theta_stride) nodes.push_back(i);
    if (nodes.back() != L - 1) nodes.push_back(L - 1);
    for (int n = 0; n < M; n += slice_stride) slices.push_back(n);
    if (slices.back() != M - 1) slices.push_back(M - 1);
    const size_t Lk = nodes.size(), Mk = slices.size();
    // the full fields through the read path, then the kept rows and columns
    std::vector<double> th(L), t(M), E(M), mu(M), C(size_t(M) * L), R(size_t(M) * L);
    struct Part {
        int32_t field;
        double* dst;
        int64_t count;
    } parts[] = {{DMFE_F_THETA, th.data(), L}, {DMFE_F_T_GRID, t.data(), M}, {DMFE_F_ENERGY, E.data(), M},
                 {DMFE_F_MU, mu.data(), M},      {DMFE_F_C, C.data(), M},      {DMFE_F_R, R.data(), M}};
    for (const Part& q : parts) {
        const size_t bytes = sizeof(double) * size_t(q.count) * (q.field == DMFE_F_C || q.field == DMFE_F_R ? L : 1);
        const dmfe_status st = dmfe_read(h, q.field, 0, q.count, q.dst, bytes, 0, nullptr);
        if (st != DMFE_OK) return st;
    }
    size_t rec_bytes = 0;
    dmfe_param_record(h, nullptr, 0, &rec_bytes);
    std::vector<char> rec(rec_bytes);
    dmfe_status st = dmfe_param_record(h, rec.data(), rec.size(), &rec_bytes);
    if (st != DMFE_OK) return st;

    std::vector<unsigned char> out;
    auto put = [&](const void* p, size_t n) {
        const unsigned char* b = static_cast<const unsigned char*>(p);
        out.insert(out.end(), b, b + n);
    };
    const char magic[8] = {'D', 'M', 'F', 'E', 'S', 'N', 'P', '1'};
    const uint32_t version = 1, header = 8 + 4 + 4 + 7 * 8;
    const int64_t hdr[6] = {L, M, theta_stride, slice_stride, int64_t(Lk), int64_t(Mk)};
    const uint64_t rb = rec.size();
    put(magic, 8);
    put(&version, 4);
    put(&header, 4);
    put(hdr, sizeof(hdr));
    put(&rb, 8);
    put(rec.data(), rec.size());
    for (int64_t i : nodes) put(&th[i], 8);
    for (int64_t n : slices) put(&t[n], 8);
    for (int64_t n : slices) put(&E[n], 8);
    for (int64_t n : slices) put(&mu[n], 8);
    for (const std::vector<double>* f : {&C, &R})
        for (int64_t n : slices)
            for (int64_t i : nodes) {
                const float v = float((*f)[size_t(n) * L + i]);
                put(&v, 4);
            }
    FILE* fp = std::fopen(path, "wb");
    if (!fp) return fail_msg(DMFE_ERR_INVALID, std::string("snapshot: cannot open ") + path + " for writing");
    const bool ok = std::fwrite(out.data(), 1, out.size(), fp) == out.size();
    const bool closed = std::fclose(fp) == 0;
    if (!ok || !closed) return fail_msg(DMFE_ERR_INVALID, std::string("snapshot: write to ") + path + " failed");
    return DMFE_OK;
}

}  // extern "C"
