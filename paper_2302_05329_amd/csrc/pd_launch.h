// Internal host-side launch interface between the C ABI and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/phenomd.h"
#include "pd_bin.h"
#include "pd_metric.h"

namespace pd {

constexpr int kNSlot = 2 + REC_N;   // (d|h), (h|h), then one moment per record entry
constexpr int kFisherSlots = 25;    // per-chunk Fisher sums (4 intrinsic directions + moments)

// Bin-chunking policy: enough wavefronts to fill the chip even for small batches.
// Side streams (default priority, one pair per host thread and device) on which the intermediate
// and inspiral launches of a three-region pass run concurrently with the merger-ringdown launch,
// so that the short launches fill the long one's tail instead of each draining the GPU in turn.
struct RegionStreams {
    int dev = -1;
    hipStream_t s[2] = {nullptr, nullptr};
    hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};
    bool ok = false;
};
RegionStreams* region_streams();

// launch(r, stream) for the phase regions r = 3, 2, 1: region 3 on s, regions 2 and 1 on the side
// streams, forked from and joined back into s by events (all on s if the side streams are missing,
// or when `concurrent` is false: then no stream or event is created or used).
template <class F>
inline void launch_regions(hipStream_t s, F&& launch, bool concurrent = true) {
    RegionStreams* rs = concurrent ? region_streams() : nullptr;
    const bool conc = rs && hipEventRecord(rs->fork, s) == hipSuccess &&
                      hipStreamWaitEvent(rs->s[0], rs->fork, 0) == hipSuccess &&
                      hipStreamWaitEvent(rs->s[1], rs->fork, 0) == hipSuccess;
    launch(3, s);
    launch(2, conc ? rs->s[0] : s);
    launch(1, conc ? rs->s[1] : s);
    if (conc) {
        (void)hipEventRecord(rs->join[0], rs->s[0]);
        (void)hipEventRecord(rs->join[1], rs->s[1]);
        (void)hipStreamWaitEvent(s, rs->join[0], 0);
        (void)hipStreamWaitEvent(s, rs->join[1], 0);
    }
}

constexpr int kOrderBuckets = 256;  // work buckets of the point ordering (one per thread of a block)

// Waves per point of a region pass: enough for about 8192 merger-ringdown waves per launch (at 4096
// points x 8033 bins, 2 chunks measured 0.167 ms per leapfrog against 0.180 with 4), at least 512
// bins per chunk, between 1 and 64.
inline int chunks_for(int64_t n, int64_t n_bins) {
    const int64_t want = (8192 + n - 1) / n;
    int64_t cap = n_bins / 512;
    if (cap < 1) cap = 1;
    int64_t c = want < cap ? want : cap;
    if (c < 1) c = 1;
    if (c > 64) c = 64;
    return static_cast<int>(c);
}

// xf (or NULL): theta is computed from the sampler's coordinates first and written to `theta`.
// tg (or NULL): the same launch also fills the per-grid tables of grid *tg into tab (from
// data and inv_psd, either of which may be NULL), on blocks of their own.
hipError_t launch_setup_value(const double* theta, int64_t n, int param, double f_ref, const double* lam,
                              double* recs, int32_t* status, hipStream_t s, const XForm* xf = nullptr,
                              const GridArgs* tg = nullptr, const double* data = nullptr,
                              const double* inv_psd = nullptr, double* tab = nullptr);
hipError_t launch_setup_theta_tangent(const double* theta, int64_t n, int param, double f_ref,
                                      const double* lam, int rows, double* tans, hipStream_t s);
hipError_t launch_setup_fit_tangent(const double* theta, int64_t n, int param, double f_ref, const double* lam,
                                    const double* recs, double* tans, hipStream_t s);
hipError_t launch_waveform(const double* recs, int64_t n, const GridArgs& g, const double* tab, int precision,
                           double* h, hipStream_t s);
// tail (gradient passes only, or NULL): the sampler's per-point tail applied by the epilogue
hipError_t launch_loglike(const double* theta, int param, const double* recs, const double* tans, int64_t n,
                          int chunks, const GridArgs& g, const double* tab, int* segs, int* order, double* partial,
                          double* lnl, double* grad, hipEvent_t before_epilogue, hipStream_t s,
                          bool concurrent = true, const PostTail* tail = nullptr);
hipError_t launch_transitions(const double* recs, int64_t n, double* out, hipStream_t s);
hipError_t launch_fisher(const double* theta, int param, const double* recs, const double* tans, int64_t n,
                         int chunks, const GridArgs& g, const double* tab, int* segs, int* order, double* partial,
                         double* F, hipStream_t s);

int posterior_check(const pd_posterior* post);
size_t posterior_ws_bytes(const pd_posterior* post, int64_t n);
size_t hmc_workspace_bytes(const pd_posterior* post, int64_t n);
size_t rwmh_workspace_bytes(const pd_posterior* post, int64_t n);
// scale: per-coordinate step [7] (chol NULL); chol: row-major lower-triangular L [7][7], steps L xi
int rwmh_step(const pd_posterior* post, int64_t n, double* x, double* logp, const double* xi, const double* u,
              const double* scale, const double* chol, int32_t* accepted, void* ws, hipStream_t s);
// concurrent: run the record tangents and two of the three region launches on side streams (created
// once per host thread and device); false keeps every launch on `s` and creates nothing.
// tail: as for launch_loglike (with grad).  xf: theta [n][7] is an output, computed from the
// sampler's coordinates by the record setup (the record tangents then start after it).
int loglike_and_grad(const double* theta, int64_t n, int param, const pd_grid* grid, const double* lambda,
                     const double* data, const double* inv_psd, int precision, double* lnl, double* grad,
                     int32_t* status, void* workspace, size_t workspace_bytes, hipStream_t s, bool tables_ready,
                     bool concurrent = true, const PostTail* tail = nullptr, const XForm* xf = nullptr);
size_t op_workspace_bytes(int op, int64_t n, int64_t n_bins);
void set_last_error(const char* msg);
int posterior_logp(const pd_posterior* post, const double* x, int64_t n, double* logp, double* grad, void* ws,
                   hipStream_t s, bool tables_ready = false);
// mass: diagonal mass matrix [7] (chol NULL); chol: row-major lower-triangular L [7][7] with inverse
// mass matrix L L^T (mass ignored)
int hmc_step(const pd_posterior* post, int64_t n, double* x, double* logp, double* grad, const double* xi,
             const double* u, int n_leapfrog, double eps, const double* mass, const double* chol, int32_t* accepted,
             double* dh, void* ws, hipStream_t s);
int independence_mh(int64_t n, double* x, double* logp, double* logq, double* grad, const double* xp,
                    const double* logp_p, const double* logq_p, const double* grad_p, const double* u,
                    int32_t* accepted, hipStream_t s);

hipError_t launch_elementary(int fn, const double* x, int64_t n, double* out, hipStream_t s);

// Detector network (pd_network.hip): 11 parameters per point, per-site geometry.
constexpr int kNetParams = 11;
constexpr int kNetJac = 13;
struct NetSite {
    double vertex[3], xarm[3], yarm[3];
};
struct NetArgs {
    int n_det;
    double gmst;
    NetSite site[PD_NETWORK_MAX_DETECTORS];
};
hipError_t launch_net_setup(const double* theta, int64_t n, int param, const NetArgs& na, double* eff, double* jac,
                            hipStream_t s);
hipError_t launch_net_combine(int64_t n, int n_det, const double* lnl_d, const double* grad_d, const int32_t* status_d,
                              const double* jac, double* lnl, double* grad, int32_t* status, hipStream_t s);
hipError_t launch_net_fisher_combine(int64_t n, int n_det, const double* F_d, const int32_t* status_d, const double* jac,
                                     double* F, int32_t* status, hipStream_t s);

constexpr int kOverlapMaxStreams = PD_OVERLAP_MAX_STREAMS;
size_t overlap_bprime_bytes(int64_t nb, int64_t ns);
hipError_t launch_overlap(const double* recs, int64_t nt, const GridArgs& g, const double* tab, const double* data,
                          int64_t ns, const double* inv_psd, double* bp, double* out, double* hh, hipStream_t s);

int64_t flow_param_count();
size_t flow_ws_bytes(int64_t n);
int flow_forward(const float* params, const double* x, int64_t n, double* z, double* logq, int mode, hipStream_t s);
int flow_sample(const float* params, const double* z, int64_t n, double* x, double* logq, int mode, hipStream_t s);
int flow_loss_grad(const float* params, const double* x, int64_t n, float* grad, double* loss, void* ws, int mode,
                   hipStream_t s);
int adam_step(float* params, const float* grad, float* m, float* v, int64_t count, double lr, double b1, double b2,
              double eps, int64_t t, hipStream_t s);

}  // namespace pd
