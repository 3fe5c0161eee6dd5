// C ABI entry points (declared in include/phenomd.h): argument validation, workspace
// carving and kernel launches.  No entry point allocates device memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/phenomd.h"
#include "pd_launch.h"
#include "pd_mismatch.h"
#include "pd_profile.h"

// ---- kernel timing ------------------------------------------------------------------------
namespace pd {
namespace {
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_ev[PD_K_COUNT];
}  // namespace

ProfRange::ProfRange(int id, hipStream_t s) : id_(id), s_(s) {
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        on_ = g_prof_on && id >= 0 && id < PD_K_COUNT;
    }
    if (on_ && hipEventCreate(&e0_) == hipSuccess) {
        if (hipEventRecord(e0_, s_) != hipSuccess) on_ = false;
    } else {
        on_ = false;
    }
}

ProfRange::~ProfRange() {
    if (!on_) return;
    hipEvent_t e1 = nullptr;
    if (hipEventCreate(&e1) != hipSuccess) return;
    if (hipEventRecord(e1, s_) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_ev[id_].emplace_back(e0_, e1);
}
}  // namespace pd

namespace {

thread_local std::string g_last_error = "no error";

int fail(int code, const char* msg) {
    g_last_error = msg;
    return code;
}

int fail_hip(hipError_t e, const char* where) {
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return PD_EHIP;
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t rec = 0, tab = 0, tan = 0, partial = 0, seg = 0, order = 0, extra = 0, total = 0;
    int chunks = 1;
};

Layout layout_for(int op, int64_t n, int64_t nb) {
    Layout L;
    const size_t N = static_cast<size_t>(n);
    size_t off = 0;
    L.rec = off;
    off = align_up(off + N * pd::REC_N * sizeof(double));
    L.tab = off;
    off = align_up(off + static_cast<size_t>(nb) * pd::T_N * sizeof(double));
    switch (op) {
        case PD_OP_WAVEFORM:
            break;
        case PD_OP_LOGLIKE:
            L.chunks = pd::chunks_for(n, nb);
            L.partial = off;
            off = align_up(off + 3 * N * L.chunks * 2 * sizeof(double));
            L.seg = off;
            off = align_up(off + 3 * N * L.chunks * pd::kSegInts * sizeof(int));
            L.order = off;
            off = align_up(off + (2 * pd::kOrderBuckets + N) * sizeof(int) + N);
            break;
        case PD_OP_LOGLIKE_GRAD:
            L.chunks = pd::chunks_for(n, nb);
            L.tan = off;
            off = align_up(off + N * 4 * pd::REC_N * sizeof(double));
            L.partial = off;
            off = align_up(off + N * L.chunks *
                                     (pd::region_row_width(1) + pd::region_row_width(2) + pd::region_row_width(3)) *
                                     sizeof(double));
            L.seg = off;
            off = align_up(off + 3 * N * L.chunks * pd::kSegInts * sizeof(int));
            L.order = off;
            off = align_up(off + (2 * pd::kOrderBuckets + N) * sizeof(int) + N);
            break;
        case PD_OP_FISHER:
            L.chunks = pd::chunks_for(n, nb);
            L.tan = off;
            off = align_up(off + N * 7 * pd::REC_N * sizeof(double));
            L.partial = off;
            off = align_up(off + 3 * N * L.chunks * pd::kFisherSlots * sizeof(double));
            L.seg = off;
            off = align_up(off + 3 * N * L.chunks * pd::kSegInts * sizeof(int));
            L.order = off;
            off = align_up(off + (2 * pd::kOrderBuckets + N) * sizeof(int) + N);
            break;
        case PD_OP_MISMATCH_GRAD:
            L.tan = off;
            off = align_up(off + N * pd::kNumFit * pd::REC_N * sizeof(double));
            L.extra = off;
            off = align_up(off + pd::mismatch_scratch_bytes(n, nb));
            break;
        default:
            break;
    }
    L.total = off;
    return L;
}

// A side stream (default priority) per host thread and device, with fork and join events: the
// record tangents of the gradient depend only on theta, so they run there while the records,
// tables and moment pass run on the caller's stream.  Without it everything runs in order on the
// caller's stream.
struct SideStream {
    int dev = -1;
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

SideStream* side_stream() {
    thread_local std::vector<SideStream> pool;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    for (auto& e : pool)
        if (e.dev == dev) return e.s ? &e : nullptr;
    SideStream e;
    e.dev = dev;
    if (hipStreamCreateWithFlags(&e.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&e.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&e.join, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        e.s = nullptr;
    }
    pool.push_back(e);
    return pool.back().s ? &pool.back() : nullptr;
}

int check_common(const double* theta, int64_t n, int param, const pd_grid* grid, const double* lambda,
                 pd::GridArgs* g) {
    if (!theta) return fail(PD_EINVAL, "theta is NULL");
    if (!lambda) return fail(PD_EINVAL, "lambda is NULL");
    if (!grid) return fail(PD_EINVAL, "grid is NULL");
    if (n <= 0) return fail(PD_EINVAL, "n must be > 0");
    if (n > (int64_t(1) << 31) / 64) return fail(PD_EINVAL, "n too large");
    if (param < 0 || param > 3) return fail(PD_EINVAL, "unknown parameterisation");
    if (!(grid->df > 0.0) || !std::isfinite(grid->df)) return fail(PD_EINVAL, "grid df must be finite and > 0");
    if (!std::isfinite(grid->f0) || grid->f0 < 0.0) return fail(PD_EINVAL, "grid f0 must be finite and >= 0");
    if (grid->n_bins <= 0) return fail(PD_EINVAL, "grid n_bins must be > 0");
    if (grid->n_bins > (int64_t(1) << 28)) return fail(PD_EINVAL, "grid n_bins must be <= 2^28");
    if (!std::isfinite(grid->f_min) || !(grid->f_min > 0.0))
        return fail(PD_EINVAL, "grid f_min must be finite and > 0");
    if (!std::isfinite(grid->f_ref) || !(grid->f_ref > 0.0))
        return fail(PD_EINVAL, "grid f_ref must be finite and > 0");
    g->f0 = grid->f0;
    g->df = grid->df;
    g->nb = grid->n_bins;
    g->fmin = grid->f_min;
    g->fref = grid->f_ref;
    return PD_OK;
}

int check_ws(int op, int64_t n, int64_t nb, void* ws, size_t ws_bytes, Layout* L) {
    *L = layout_for(op, n, nb);
    if (!ws) return fail(PD_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return fail(PD_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < L->total) return fail(PD_ENOMEM, "workspace too small (see pd_workspace_bytes)");
    return PD_OK;
}

template <class T>
T* at(void* ws, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

}  // namespace

extern "C" {

size_t pd_workspace_bytes(int op, int64_t n, int64_t n_bins) {
    if (n <= 0 || n_bins <= 0 || op < 0 || op > PD_OP_MISMATCH_GRAD) return 0;
    return layout_for(op, n, n_bins).total;
}

}  // extern "C"

size_t pd::op_workspace_bytes(int op, int64_t n, int64_t n_bins) { return pd_workspace_bytes(op, n, n_bins); }
void pd::set_last_error(const char* msg) { g_last_error = msg; }

extern "C" {

const char* pd_last_error(void) { return g_last_error.c_str(); }

int pd_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(pd::g_prof_mu);
    pd::g_prof_on = (on != 0);
    return PD_OK;
}

int pd_profile_read(int kernel, double* total_ms, int64_t* launches) {
    if (kernel < 0 || kernel >= PD_K_COUNT) return fail(PD_EINVAL, "unknown kernel id");
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    {
        std::lock_guard<std::mutex> lk(pd::g_prof_mu);
        ev.swap(pd::g_prof_ev[kernel]);
    }
    double sum = 0.0;
    int rc = PD_OK;
    for (auto& pr : ev) {
        float ms = 0.0f;
        if (hipEventSynchronize(pr.second) != hipSuccess || hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess)
            rc = fail(PD_EHIP, "event timing failed");
        sum += ms;
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    if (total_ms) *total_ms = sum;
    if (launches) *launches = static_cast<int64_t>(ev.size());
    return rc;
}

const char* pd_version(void) { return "phenomd-mi355x 0.1 (gfx950)"; }

int pd_waveform_eval(const double* theta, int64_t n, int param, const pd_grid* grid, const double* lambda,
                     int precision, double* h_out, int32_t* status, void* workspace, size_t workspace_bytes,
                     void* stream) {
    pd::GridArgs g;
    int rc = check_common(theta, n, param, grid, lambda, &g);
    if (rc) return rc;
    if (!h_out) return fail(PD_EINVAL, "h_out is NULL");
    if (precision == PD_MIXED) return fail(PD_EUNSUPPORTED, "PD_MIXED (FP32 amplitude) is not implemented; use PD_FP64");
    if (precision != PD_FP64) return fail(PD_EINVAL, "unknown precision");
    Layout L;
    rc = check_ws(PD_OP_WAVEFORM, n, g.nb, workspace, workspace_bytes, &L);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* recs = at<double>(workspace, L.rec);
    double* tab = at<double>(workspace, L.tab);
    // records and grid tables in one launch
    hipError_t e = pd::launch_setup_value(theta, n, param, g.fref, lambda, recs, status, s, nullptr, &g, nullptr,
                                          nullptr, tab);
    if (e != hipSuccess) return fail_hip(e, "setup");
    e = pd::launch_waveform(recs, n, g, tab, precision, h_out, s);
    if (e != hipSuccess) return fail_hip(e, "waveform");
    return PD_OK;
}

int pd_loglike_and_grad(const double* theta, int64_t n, int param, const pd_grid* grid, const double* lambda,
                        const double* data, const double* inv_psd, int precision, double* lnl, double* grad,
                        int32_t* status, void* workspace, size_t workspace_bytes, void* stream) {
    return pd::loglike_and_grad(theta, n, param, grid, lambda, data, inv_psd, precision, lnl, grad, status, workspace,
                                workspace_bytes, static_cast<hipStream_t>(stream), false);
}

}  // extern "C"

// tables_ready: the workspace already holds this grid's tables for the same data and noise
// weights (a caller that evaluates many parameter batches against one data set, such as the
// leapfrog steps of one HMC transition, computes them once).
int pd::loglike_and_grad(const double* theta, int64_t n, int param, const pd_grid* grid, const double* lambda,
                         const double* data, const double* inv_psd, int precision, double* lnl, double* grad,
                         int32_t* status, void* workspace, size_t workspace_bytes, hipStream_t s,
                         bool tables_ready, bool concurrent, const pd::PostTail* tail, const pd::XForm* xf) {
    pd::GridArgs g;
    int rc = check_common(theta, n, param, grid, lambda, &g);
    if (rc) return rc;
    if (!data) return fail(PD_EINVAL, "data is NULL");
    if (!inv_psd) return fail(PD_EINVAL, "inv_psd is NULL");
    if (!lnl) return fail(PD_EINVAL, "lnl is NULL");
    if (precision == PD_MIXED) return fail(PD_EUNSUPPORTED, "PD_MIXED (FP32 amplitude) is not implemented; use PD_FP64");
    if (precision != PD_FP64) return fail(PD_EINVAL, "unknown precision");
    const int op = grad ? PD_OP_LOGLIKE_GRAD : PD_OP_LOGLIKE;
    Layout L;
    rc = check_ws(op, n, g.nb, workspace, workspace_bytes, &L);
    if (rc) return rc;
    double* recs = at<double>(workspace, L.rec);
    double* partial = at<double>(workspace, L.partial);
    double* tab = at<double>(workspace, L.tab);
    double* tans = grad ? at<double>(workspace, L.tan) : nullptr;
    hipError_t e = hipSuccess;
    SideStream* side = (grad && concurrent) ? side_stream() : nullptr;
    // the record tangents run on the side stream, concurrently with the records and the pass (after
    // the records when those compute theta from the sampler's coordinates)
    auto launch_tangents = [&]() -> int {
        hipStream_t ts = s;
        if (side && hipEventRecord(side->fork, s) == hipSuccess && hipStreamWaitEvent(side->s, side->fork, 0) == hipSuccess)
            ts = side->s;
        else
            side = nullptr;
        e = pd::launch_setup_theta_tangent(theta, n, param, g.fref, lambda, 4, tans, ts);
        if (e != hipSuccess) return fail_hip(e, "setup tangents");
        if (side && hipEventRecord(side->join, side->s) != hipSuccess) return fail_hip(hipGetLastError(), "join");
        return PD_OK;
    };
    if (grad && !xf) {
        rc = launch_tangents();
        if (rc) return rc;
    }
    // a failure past this point still joins the side stream, so that no kernel of this call
    // writes into the workspace after the error is returned
    auto fail_joined = [&](hipError_t err, const char* what) {
        if (side) (void)hipStreamWaitEvent(s, side->join, 0);
        return fail_hip(err, what);
    };
    // records and (unless already built) grid tables in one launch
    e = pd::launch_setup_value(theta, n, param, g.fref, lambda, recs, status, s, xf, tables_ready ? nullptr : &g,
                               data, inv_psd, tab);
    if (e != hipSuccess) return fail_joined(e, "setup");
    if (grad && xf) {
        rc = launch_tangents();
        if (rc) return rc;
    }
    e = pd::launch_loglike(theta, param, recs, tans, n, L.chunks, g, tab, at<int>(workspace, L.seg),
                           at<int>(workspace, L.order), partial, lnl,
                           grad, side ? side->join : nullptr, s, concurrent, grad ? tail : nullptr);
    if (e != hipSuccess) return fail_joined(e, "loglike");
    return PD_OK;
}

extern "C" {

int pd_fisher(const double* theta, int64_t n, int param, const pd_grid* grid, const double* lambda,
              const double* inv_psd, double* F, int32_t* status, void* workspace, size_t workspace_bytes,
              void* stream) {
    pd::GridArgs g;
    int rc = check_common(theta, n, param, grid, lambda, &g);
    if (rc) return rc;
    if (!inv_psd) return fail(PD_EINVAL, "inv_psd is NULL");
    if (!F || !inv_psd) return fail(PD_EINVAL, "NULL argument");
    Layout L;
    rc = check_ws(PD_OP_FISHER, n, g.nb, workspace, workspace_bytes, &L);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* recs = at<double>(workspace, L.rec);
    double* tans = at<double>(workspace, L.tan);
    double* partial = at<double>(workspace, L.partial);
    double* tab = at<double>(workspace, L.tab);
    // records and grid tables in one launch
    hipError_t e = pd::launch_setup_value(theta, n, param, g.fref, lambda, recs, status, s, nullptr, &g, nullptr,
                                          inv_psd, tab);
    if (e != hipSuccess) return fail_hip(e, "setup");
    e = pd::launch_setup_theta_tangent(theta, n, param, g.fref, lambda, 7, tans, s);
    if (e != hipSuccess) return fail_hip(e, "setup tangents");
    e = pd::launch_fisher(theta, param, recs, tans, n, L.chunks, g, tab, at<int>(workspace, L.seg),
                          at<int>(workspace, L.order), partial, F, s);
    if (e != hipSuccess) return fail_hip(e, "fisher");
    return PD_OK;
}

int pd_transition_frequencies(const double* theta, int64_t n, int param, const pd_grid* grid, const double* lambda,
                              double* out, void* workspace, size_t workspace_bytes, void* stream) {
    pd::GridArgs g;
    int rc = check_common(theta, n, param, grid, lambda, &g);
    if (rc) return rc;
    if (!out) return fail(PD_EINVAL, "out is NULL");
    Layout L;
    rc = check_ws(PD_OP_WAVEFORM, n, g.nb, workspace, workspace_bytes, &L);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* recs = at<double>(workspace, L.rec);
    hipError_t e = pd::launch_setup_value(theta, n, param, g.fref, lambda, recs, nullptr, s);
    if (e != hipSuccess) return fail_hip(e, "setup");
    e = pd::launch_transitions(recs, n, out, s);
    if (e != hipSuccess) return fail_hip(e, "transitions");
    return PD_OK;
}

int pd_mismatch_grad(const double* theta, int64_t nt, int param, const pd_grid* grid, const double* lambda,
                     const double* targets, const double* inv_psd, double* mismatch, double* dsum_dlambda,
                     int32_t* lag, void* workspace, size_t workspace_bytes, void* stream) {
    pd::GridArgs g;
    int rc = check_common(theta, nt, param, grid, lambda, &g);
    if (rc) return rc;
    if (!targets) return fail(PD_EINVAL, "targets is NULL");
    if (!inv_psd) return fail(PD_EINVAL, "inv_psd is NULL");
    if (!mismatch) return fail(PD_EINVAL, "mismatch is NULL");
    if ((g.nb & (g.nb - 1)) != 0 || g.nb < (int64_t(1) << pd::kFFTMinLog2) || g.nb > (int64_t(1) << pd::kFFTMaxLog2))
        return fail(PD_EUNSUPPORTED, "mismatch needs n_bins = 2^n, 6 <= n <= 16 (the FFT length)");
    Layout L;
    rc = check_ws(PD_OP_MISMATCH_GRAD, nt, g.nb, workspace, workspace_bytes, &L);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* recs = at<double>(workspace, L.rec);
    double* tans = at<double>(workspace, L.tan);
    void* scratch = at<void>(workspace, L.extra);
    double* tab = at<double>(workspace, L.tab);
    // records and grid tables in one launch
    hipError_t e = pd::launch_setup_value(theta, nt, param, g.fref, lambda, recs, nullptr, s, nullptr, &g, nullptr,
                                          inv_psd, tab);
    if (e != hipSuccess) return fail_hip(e, "setup");
    if (dsum_dlambda) {
        e = pd::launch_setup_fit_tangent(theta, nt, param, g.fref, lambda, recs, tans, s);
        if (e != hipSuccess) return fail_hip(e, "setup fit tangents");
    }
    e = pd::launch_mismatch(recs, dsum_dlambda ? tans : nullptr, nt, g, tab, targets, inv_psd, scratch, mismatch,
                            dsum_dlambda, lag, s);
    if (e != hipSuccess) return fail_hip(e, "mismatch");
    return PD_OK;
}

}  // extern "C"

namespace {

struct NetLayout {
    size_t ll = 0, eff = 0, jac = 0, lnl = 0, grad = 0, status = 0, total = 0;
};

// Network workspace: the single-site workspace of `op` (reused by every site in turn), then per
// (site, point) the effective rows, their derivatives, and the site results (ln L in `lnl` and
// the gradient in `grad` for PD_OP_LOGLIKE_GRAD; the 7x7 Fisher matrix in `grad` for PD_OP_FISHER).
NetLayout net_layout(int64_t n, int64_t nb, int n_det, int op = PD_OP_LOGLIKE_GRAD) {
    NetLayout L;
    const size_t M = static_cast<size_t>(n) * static_cast<size_t>(n_det);
    size_t off = align_up(layout_for(op, n, nb).total);
    L.eff = off;
    off = align_up(off + M * 7 * sizeof(double));
    L.jac = off;
    off = align_up(off + M * pd::kNetJac * sizeof(double));
    L.lnl = off;
    off = align_up(off + M * sizeof(double));
    L.grad = off;
    off = align_up(off + M * (op == PD_OP_FISHER ? 49 : 7) * sizeof(double));
    L.status = off;
    off = align_up(off + M * sizeof(int32_t));
    L.total = off;
    return L;
}

}  // namespace

extern "C" {

size_t pd_network_workspace_bytes(int64_t n, int64_t n_bins, int n_det) {
    if (n <= 0 || n_bins <= 0 || n_det < 1 || n_det > PD_NETWORK_MAX_DETECTORS) return 0;
    return net_layout(n, n_bins, n_det).total;
}

}  // extern "C"

namespace {

int net_check(const double* theta, int64_t n, int param, const pd_grid* grid, const double* lambda, int n_det,
              const pd_detector* detectors, double gmst, pd::GridArgs* g, pd::NetArgs* na) {
    int rc = check_common(theta, n, param, grid, lambda, g);
    if (rc) return rc;
    if (n_det < 1 || n_det > PD_NETWORK_MAX_DETECTORS) return fail(PD_EINVAL, "n_det out of range");
    if (!detectors) return fail(PD_EINVAL, "detectors is NULL");
    if (!std::isfinite(gmst)) return fail(PD_EINVAL, "gmst must be finite");
    na->n_det = n_det;
    na->gmst = gmst;
    for (int d = 0; d < n_det; ++d)
        for (int k = 0; k < 3; ++k) {
            const double v[3] = {detectors[d].vertex[k], detectors[d].xarm[k], detectors[d].yarm[k]};
            if (!std::isfinite(v[0]) || !std::isfinite(v[1]) || !std::isfinite(v[2]))
                return fail(PD_EINVAL, "detector geometry must be finite");
            na->site[d].vertex[k] = v[0];
            na->site[d].xarm[k] = v[1];
            na->site[d].yarm[k] = v[2];
        }
    return PD_OK;
}

}  // namespace

extern "C" {

int pd_network_loglike_and_grad(const double* theta, int64_t n, int param, const pd_grid* grid, const double* lambda,
                                int n_det, const pd_detector* detectors, double gmst, const double* data,
                                const double* inv_psd, double* lnl, double* grad, int32_t* status, void* workspace,
                                size_t workspace_bytes, void* stream) {
    pd::GridArgs g;
    pd::NetArgs na;
    int rc = net_check(theta, n, param, grid, lambda, n_det, detectors, gmst, &g, &na);
    if (rc) return rc;
    if (!data || !inv_psd || !lnl) return fail(PD_EINVAL, "NULL argument");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(PD_EINVAL, "bad workspace");
    const NetLayout L = net_layout(n, g.nb, n_det);
    if (workspace_bytes < L.total) return fail(PD_ENOMEM, "workspace too small (see pd_network_workspace_bytes)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* eff = at<double>(workspace, L.eff);
    double* jac = at<double>(workspace, L.jac);
    double* lnl_d = at<double>(workspace, L.lnl);
    double* grad_d = at<double>(workspace, L.grad);
    int32_t* st_d = at<int32_t>(workspace, L.status);
    hipError_t e = pd::launch_net_setup(theta, n, param, na, eff, jac, s);
    if (e != hipSuccess) return fail_hip(e, "network setup");
    const size_t ll_bytes = layout_for(PD_OP_LOGLIKE_GRAD, n, g.nb).total;
    for (int d = 0; d < n_det; ++d) {
        const int64_t off = static_cast<int64_t>(d) * n;
        rc = pd::loglike_and_grad(eff + off * 7, n, param, grid, lambda, data + static_cast<int64_t>(d) * g.nb * 2,
                                  inv_psd + static_cast<int64_t>(d) * g.nb, PD_FP64, lnl_d + off,
                                  grad ? grad_d + off * 7 : nullptr, st_d + off, at<void>(workspace, L.ll), ll_bytes,
                                  s, false);
        if (rc != PD_OK) return rc;
    }
    e = pd::launch_net_combine(n, n_det, lnl_d, grad_d, st_d, jac, lnl, grad, status, s);
    if (e != hipSuccess) return fail_hip(e, "network combine");
    return PD_OK;
}

size_t pd_network_strain_workspace_bytes(int64_t n, int64_t n_bins) {
    if (n <= 0 || n_bins <= 0) return 0;
    return net_layout(n, n_bins, 1, PD_OP_WAVEFORM).total;
}

int pd_network_strain(const double* theta, int64_t n, int param, const pd_grid* grid, const double* lambda,
                      const pd_detector* detector, double gmst, double* h_out, int32_t* status, void* workspace,
                      size_t workspace_bytes, void* stream) {
    pd::GridArgs g;
    pd::NetArgs na;
    int rc = net_check(theta, n, param, grid, lambda, 1, detector, gmst, &g, &na);
    if (rc) return rc;
    if (!h_out) return fail(PD_EINVAL, "h_out is NULL");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(PD_EINVAL, "bad workspace");
    const NetLayout L = net_layout(n, g.nb, 1, PD_OP_WAVEFORM);
    if (workspace_bytes < L.total) return fail(PD_ENOMEM, "workspace too small (see pd_network_strain_workspace_bytes)");
    double* eff = at<double>(workspace, L.eff);
    hipError_t e = pd::launch_net_setup(theta, n, param, na, eff, at<double>(workspace, L.jac),
                                        static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "network setup");
    return pd_waveform_eval(eff, n, param, grid, lambda, PD_FP64, h_out, status, workspace,
                            layout_for(PD_OP_WAVEFORM, n, g.nb).total, stream);
}

size_t pd_network_fisher_workspace_bytes(int64_t n, int64_t n_bins, int n_det) {
    if (n <= 0 || n_bins <= 0 || n_det < 1 || n_det > PD_NETWORK_MAX_DETECTORS) return 0;
    return net_layout(n, n_bins, n_det, PD_OP_FISHER).total;
}

int pd_network_fisher(const double* theta, int64_t n, int param, const pd_grid* grid, const double* lambda, int n_det,
                      const pd_detector* detectors, double gmst, const double* inv_psd, double* F, int32_t* status,
                      void* workspace, size_t workspace_bytes, void* stream) {
    pd::GridArgs g;
    pd::NetArgs na;
    int rc = net_check(theta, n, param, grid, lambda, n_det, detectors, gmst, &g, &na);
    if (rc) return rc;
    if (!F) return fail(PD_EINVAL, "F is NULL");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(PD_EINVAL, "bad workspace");
    const NetLayout L = net_layout(n, g.nb, n_det, PD_OP_FISHER);
    if (workspace_bytes < L.total) return fail(PD_ENOMEM, "workspace too small (see pd_network_fisher_workspace_bytes)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* eff = at<double>(workspace, L.eff);
    double* jac = at<double>(workspace, L.jac);
    double* F_d = at<double>(workspace, L.grad);
    int32_t* st_d = at<int32_t>(workspace, L.status);
    hipError_t e = pd::launch_net_setup(theta, n, param, na, eff, jac, s);
    if (e != hipSuccess) return fail_hip(e, "network setup");
    const size_t f_bytes = layout_for(PD_OP_FISHER, n, g.nb).total;
    for (int d = 0; d < n_det; ++d) {
        const int64_t off = static_cast<int64_t>(d) * n;
        rc = pd_fisher(eff + off * 7, n, param, grid, lambda, inv_psd + static_cast<int64_t>(d) * g.nb, F_d + off * 49,
                       st_d + off, workspace, f_bytes, stream);
        if (rc != PD_OK) return rc;
    }
    e = pd::launch_net_fisher_combine(n, n_det, F_d, st_d, jac, F, status, s);
    if (e != hipSuccess) return fail_hip(e, "network Fisher combine");
    return PD_OK;
}

int pd_fit_lambda_step(const double* theta, int64_t nt, int param, const pd_grid* grid, double* lambda,
                       const double* targets, const double* inv_psd, double alpha, const double* precond,
                       double* mismatch, double* dsum_dlambda, void* workspace, size_t workspace_bytes,
                       void* stream) {
    if (!dsum_dlambda) return fail(PD_EINVAL, "dsum_dlambda is NULL");
    if (dsum_dlambda == lambda) return fail(PD_EINVAL, "dsum_dlambda must not alias lambda");
    if (precond && (precond == lambda || precond == dsum_dlambda))
        return fail(PD_EINVAL, "precond must not alias lambda or dsum_dlambda");
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(PD_EINVAL, "alpha must be finite and >= 0");
    const int rc = pd_mismatch_grad(theta, nt, param, grid, lambda, targets, inv_psd, mismatch, dsum_dlambda,
                                    nullptr, workspace, workspace_bytes, stream);
    if (rc != PD_OK) return rc;
    const hipError_t e = pd::launch_lambda_update(lambda, dsum_dlambda, precond, alpha / static_cast<double>(nt),
                                                  static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "coefficient update");
    return PD_OK;
}

}  // extern "C"

namespace {

int hmc_common(const pd_posterior* post, int64_t n, double* x, double* logp, double* grad, const double* xi,
               const double* u, int n_leapfrog, double eps, const double* mass, const double* chol, int32_t* accepted,
               double* dh, void* workspace, size_t workspace_bytes, void* stream) {
    if (pd::posterior_check(post) != PD_OK) return fail(PD_EINVAL, "invalid posterior description");
    if (!x || !logp || !grad || !xi || !u) return fail(PD_EINVAL, "NULL argument");
    if (n <= 0 || n > (int64_t(1) << 31) / 64) return fail(PD_EINVAL, "bad n");
    if (n_leapfrog < 1 || n_leapfrog > 100000) return fail(PD_EINVAL, "n_leapfrog out of range");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(PD_EINVAL, "eps must be finite and > 0");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(PD_EINVAL, "bad workspace");
    if (workspace_bytes < pd::hmc_workspace_bytes(post, n)) return fail(PD_ENOMEM, "workspace too small");
    const int rc = pd::hmc_step(post, n, x, logp, grad, xi, u, n_leapfrog, eps, mass, chol, accepted, dh, workspace,
                                static_cast<hipStream_t>(stream));
    if (rc != PD_OK) return fail(rc, "hmc step failed");
    return PD_OK;
}

int rwmh_common(const pd_posterior* post, int64_t n, double* x, double* logp, const double* xi, const double* u,
                const double* scale, const double* chol, int32_t* accepted, void* workspace, size_t workspace_bytes,
                void* stream) {
    if (pd::posterior_check(post) != PD_OK) return fail(PD_EINVAL, "invalid posterior description");
    if (!x || !logp || !xi || !u) return fail(PD_EINVAL, "NULL argument");
    if (n <= 0 || n > (int64_t(1) << 31) / 64) return fail(PD_EINVAL, "bad n");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(PD_EINVAL, "bad workspace");
    if (workspace_bytes < pd::rwmh_workspace_bytes(post, n)) return fail(PD_ENOMEM, "workspace too small");
    const int rc = pd::rwmh_step(post, n, x, logp, xi, u, scale, chol, accepted, workspace,
                                 static_cast<hipStream_t>(stream));
    if (rc != PD_OK) return fail(rc, "random-walk step failed");
    return PD_OK;
}

}  // namespace

extern "C" {

size_t pd_posterior_workspace_bytes(const pd_posterior* post, int64_t n) {
    if (pd::posterior_check(post) != PD_OK || n <= 0) return 0;
    return pd::posterior_ws_bytes(post, n);
}

size_t pd_hmc_workspace_bytes(const pd_posterior* post, int64_t n) {
    if (pd::posterior_check(post) != PD_OK || n <= 0) return 0;
    return pd::hmc_workspace_bytes(post, n);
}

int pd_posterior_logp(const pd_posterior* post, const double* x, int64_t n, double* logp, double* grad,
                      void* workspace, size_t workspace_bytes, void* stream) {
    if (pd::posterior_check(post) != PD_OK) return fail(PD_EINVAL, "invalid posterior description");
    if (!x || !logp) return fail(PD_EINVAL, "x or logp is NULL");
    if (n <= 0 || n > (int64_t(1) << 31) / 64) return fail(PD_EINVAL, "bad n");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(PD_EINVAL, "bad workspace");
    if (workspace_bytes < pd::posterior_ws_bytes(post, n)) return fail(PD_ENOMEM, "workspace too small");
    const int rc = pd::posterior_logp(post, x, n, logp, grad, workspace, static_cast<hipStream_t>(stream));
    if (rc != PD_OK) return fail(rc, "posterior evaluation failed");
    return PD_OK;
}

int pd_hmc_step(const pd_posterior* post, int64_t n, double* x, double* logp, double* grad, const double* xi,
                const double* u, int n_leapfrog, double eps, const double* mass, int32_t* accepted, double* dh,
                void* workspace, size_t workspace_bytes, void* stream) {
    if (!mass) return fail(PD_EINVAL, "NULL argument");
    for (int j = 0; j < 7; ++j)
        if (!(mass[j] > 0.0) || !std::isfinite(mass[j])) return fail(PD_EINVAL, "mass must be finite and > 0");
    return hmc_common(post, n, x, logp, grad, xi, u, n_leapfrog, eps, mass, nullptr, accepted, dh, workspace,
                      workspace_bytes, stream);
}

int pd_hmc_step_dense(const pd_posterior* post, int64_t n, double* x, double* logp, double* grad, const double* xi,
                      const double* u, int n_leapfrog, double eps, const double* chol, int32_t* accepted, double* dh,
                      void* workspace, size_t workspace_bytes, void* stream) {
    if (!chol) return fail(PD_EINVAL, "NULL argument");
    for (int j = 0; j < 7; ++j) {
        if (!(chol[j * 7 + j] > 0.0)) return fail(PD_EINVAL, "chol must have a positive diagonal");
        for (int k = 0; k <= j; ++k)
            if (!std::isfinite(chol[j * 7 + k])) return fail(PD_EINVAL, "chol must be finite");
    }
    return hmc_common(post, n, x, logp, grad, xi, u, n_leapfrog, eps, nullptr, chol, accepted, dh, workspace,
                      workspace_bytes, stream);
}

size_t pd_rwmh_workspace_bytes(const pd_posterior* post, int64_t n) {
    if (pd::posterior_check(post) != PD_OK || n <= 0) return 0;
    return pd::rwmh_workspace_bytes(post, n);
}

int pd_rwmh_step(const pd_posterior* post, int64_t n, double* x, double* logp, const double* xi, const double* u,
                 const double* scale, int32_t* accepted, void* workspace, size_t workspace_bytes, void* stream) {
    if (!scale) return fail(PD_EINVAL, "NULL argument");
    for (int j = 0; j < 7; ++j)
        if (!(scale[j] >= 0.0) || !std::isfinite(scale[j])) return fail(PD_EINVAL, "scale must be finite and >= 0");
    return rwmh_common(post, n, x, logp, xi, u, scale, nullptr, accepted, workspace, workspace_bytes, stream);
}

int pd_rwmh_step_dense(const pd_posterior* post, int64_t n, double* x, double* logp, const double* xi,
                       const double* u, const double* chol, int32_t* accepted, void* workspace, size_t workspace_bytes,
                       void* stream) {
    if (!chol) return fail(PD_EINVAL, "NULL argument");
    for (int j = 0; j < 7; ++j)
        for (int k = 0; k <= j; ++k)
            if (!std::isfinite(chol[j * 7 + k])) return fail(PD_EINVAL, "chol must be finite");
    return rwmh_common(post, n, x, logp, xi, u, nullptr, chol, accepted, workspace, workspace_bytes, stream);
}

int pd_independence_mh(int64_t n, double* x, double* logp, double* logq, double* grad, const double* xp,
                       const double* logp_p, const double* logq_p, const double* grad_p, const double* u,
                       int32_t* accepted, void* stream) {
    if (!x || !logp || !logq || !xp || !logp_p || !logq_p || !u) return fail(PD_EINVAL, "NULL argument");
    if ((grad == nullptr) != (grad_p == nullptr)) return fail(PD_EINVAL, "grad and grad_p must both be set or NULL");
    if (n <= 0 || n > (int64_t(1) << 31) / 64) return fail(PD_EINVAL, "bad n");
    const int rc = pd::independence_mh(n, x, logp, logq, grad, xp, logp_p, logq_p, grad_p, u, accepted,
                                       static_cast<hipStream_t>(stream));
    if (rc != PD_OK) return fail(rc, "independence MH failed");
    return PD_OK;
}

size_t pd_overlap_workspace_bytes(int64_t nt, int64_t ns, int64_t n_bins) {
    if (nt <= 0 || ns <= 0 || ns > PD_OVERLAP_MAX_STREAMS || n_bins <= 0) return 0;
    const Layout L = layout_for(PD_OP_WAVEFORM, nt, n_bins);
    return align_up(L.total + pd::overlap_bprime_bytes(n_bins, ns));
}

int pd_overlap(const double* theta, int64_t nt, int param, const pd_grid* grid, const double* lambda,
               const double* data, int64_t ns, const double* inv_psd, double* overlap, double* hh,
               int32_t* status, void* workspace, size_t workspace_bytes, void* stream) {
    pd::GridArgs g;
    int rc = check_common(theta, nt, param, grid, lambda, &g);
    if (rc) return rc;
    if (!data) return fail(PD_EINVAL, "data is NULL");
    if (!inv_psd) return fail(PD_EINVAL, "inv_psd is NULL");
    if (!overlap) return fail(PD_EINVAL, "overlap is NULL");
    if (ns <= 0 || ns > PD_OVERLAP_MAX_STREAMS) return fail(PD_EINVAL, "ns must be in [1, 64]");
    Layout L;
    rc = check_ws(PD_OP_WAVEFORM, nt, g.nb, workspace, workspace_bytes, &L);
    if (rc) return rc;
    if (workspace_bytes < pd_overlap_workspace_bytes(nt, ns, g.nb))
        return fail(PD_ENOMEM, "workspace too small (see pd_overlap_workspace_bytes)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* recs = at<double>(workspace, L.rec);
    double* tab = at<double>(workspace, L.tab);
    double* bp = at<double>(workspace, L.total);
    // records and grid tables in one launch
    hipError_t e = pd::launch_setup_value(theta, nt, param, g.fref, lambda, recs, status, s, nullptr, &g, nullptr,
                                          inv_psd, tab);
    if (e != hipSuccess) return fail_hip(e, "setup");
    e = pd::launch_overlap(recs, nt, g, tab, data, ns, inv_psd, bp, overlap, hh, s);
    if (e != hipSuccess) return fail_hip(e, "overlap");
    return PD_OK;
}

int pd_elementary_eval(int fn, const double* x, int64_t n, double* out, void* stream) {
    if (!x || !out) return fail(PD_EINVAL, "NULL argument");
    if (fn < PD_FN_SIN || fn > PD_FN_ATAN_TABLE) return fail(PD_EINVAL, "unknown function");
    if (n <= 0 || n > (int64_t(1) << 31)) return fail(PD_EINVAL, "bad n");
    if (pd::launch_elementary(fn, x, n, out, static_cast<hipStream_t>(stream)) != hipSuccess)
        return fail(PD_EHIP, "launch failed");
    return PD_OK;
}

int64_t pd_flow_param_count(void) { return pd::flow_param_count(); }

size_t pd_flow_workspace_bytes(int64_t n) { return n > 0 ? pd::flow_ws_bytes(n) : 0; }

int pd_flow_forward(const float* params, const double* x, int64_t n, double* z, double* logq, int mode,
                    void* stream) {
    if (!params || !x || !logq) return fail(PD_EINVAL, "NULL argument");
    if (mode != PD_FLOW_FP32 && mode != PD_FLOW_BF16) return fail(PD_EINVAL, "unknown flow mode");
    if (n <= 0 || n > (int64_t(1) << 31) / 64) return fail(PD_EINVAL, "bad n");
    const int rc = pd::flow_forward(params, x, n, z, logq, mode, static_cast<hipStream_t>(stream));
    return rc == PD_OK ? PD_OK : fail(rc, "flow forward failed");
}

int pd_flow_sample(const float* params, const double* z, int64_t n, double* x, double* logq, int mode,
                   void* stream) {
    if (!params || !z || !x || !logq) return fail(PD_EINVAL, "NULL argument");
    if (mode != PD_FLOW_FP32 && mode != PD_FLOW_BF16) return fail(PD_EINVAL, "unknown flow mode");
    if (n <= 0 || n > (int64_t(1) << 31) / 64) return fail(PD_EINVAL, "bad n");
    const int rc = pd::flow_sample(params, z, n, x, logq, mode, static_cast<hipStream_t>(stream));
    return rc == PD_OK ? PD_OK : fail(rc, "flow sample failed");
}

int pd_flow_loss_grad(const float* params, const double* x, int64_t n, float* grad, double* loss, void* workspace,
                      size_t workspace_bytes, int mode, void* stream) {
    if (!params || !x || !grad) return fail(PD_EINVAL, "NULL argument");
    if (mode != PD_FLOW_FP32 && mode != PD_FLOW_BF16) return fail(PD_EINVAL, "unknown flow mode");
    if (n <= 0 || n > (int64_t(1) << 31) / 64) return fail(PD_EINVAL, "bad n");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(PD_EINVAL, "bad workspace");
    if (workspace_bytes < pd::flow_ws_bytes(n)) return fail(PD_ENOMEM, "workspace too small");
    const int rc = pd::flow_loss_grad(params, x, n, grad, loss, workspace, mode, static_cast<hipStream_t>(stream));
    return rc == PD_OK ? PD_OK : fail(rc, "flow gradient failed");
}

int pd_adam_step(float* params, const float* grad, float* m, float* v, int64_t count, double lr, double beta1,
                 double beta2, double eps, int64_t t, void* stream) {
    if (!params || !grad || !m || !v) return fail(PD_EINVAL, "NULL argument");
    if (count <= 0 || t < 1) return fail(PD_EINVAL, "bad count or step");
    if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
        return fail(PD_EINVAL, "bad Adam hyper-parameters");
    const int rc = pd::adam_step(params, grad, m, v, count, lr, beta1, beta2, eps, t, static_cast<hipStream_t>(stream));
    return rc == PD_OK ? PD_OK : fail(rc, "adam failed");
}

}  // extern "C"
