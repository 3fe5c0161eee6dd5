// Samplers on the GPU (paper Sec. 3.3): posterior log-density and gradient in
// unconstrained coordinates, Hamiltonian Monte Carlo with a dense (or diagonal) metric, the
// random-walk Metropolis-Hastings baseline the paper compares it with (Gaussian steps), and
// the Metropolis-Hastings accept step of an independence proposal (the learned flow).
//
// Coordinates.  The sampler moves x in R^7.  For the gravitational-wave targets (one detector, or
// a network of sites with the orientation and sky position held fixed) the
// source parameters are theta = (Mc, q, chi1, chi2, D, tc, phic) with
//   theta_i = lo_i + (hi_i - lo_i) * sigmoid(x_i)   (bounded uniform priors; for phic an
//   interval of length pi is one full period of the likelihood),
// so log pi(x) = lnL(theta(x)) + sum_i log(dtheta_i/dx_i).  The Gaussian target
// (independent normals) exists to test the sampler machinery against a known answer.
//
// Random numbers are inputs (momentum draws, uniforms for the accept test): every call
// is a deterministic function of its arguments.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/phenomd.h"
#include "pd_launch.h"
#include "pd_metric.h"

namespace pd {

namespace {

__device__ __forceinline__ double sigmoid(double x) {
    return (x >= 0.0) ? 1.0 / (1.0 + exp(-x)) : exp(x) / (1.0 + exp(x));
}

// x -> theta, d theta / d x, and the log-Jacobian with its derivative.  DRIFT: first the leapfrog
// drift x += eps L r (x updated in place).
struct Drift {
    double eps;
    Metric m;
    const double* p;
};

template <bool DRIFT>
__global__ void k_transform(double* __restrict__ x, int64_t n, pd_posterior post, double* __restrict__ theta,
                            double* __restrict__ dtdx, double* __restrict__ lj, double* __restrict__ dlj, Drift dr,
                            int ts) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // ts = 11: network rows, the fixed orientation appended after the 7 sampled parameters
    if (ts == 11)
        for (int k = 0; k < 4; ++k) theta[i * 11 + 7 + k] = post.orient[k];
    double acc = 0.0;
    double dx[7];
    if (DRIFT) metric_drift(dr.m, dr.eps, dr.p + i * 7, dx);
    for (int j = 0; j < 7; ++j) {
        double xv = x[i * 7 + j];
        if (DRIFT) {
            xv += dx[j];
            x[i * 7 + j] = xv;
        }
        const double s = sigmoid(xv);
        const double w = post.hi[j] - post.lo[j];
        theta[i * ts + j] = post.lo[j] + w * s;
        const double d = w * s * (1.0 - s);
        dtdx[i * 7 + j] = d;
        // log(w s (1-s)) = log w - softplus(-x) - softplus(x)
        const double ax = fabs(xv);
        acc += log(w) - ax - 2.0 * log1p(exp(-ax));
        dlj[i * 7 + j] = 1.0 - 2.0 * s;
    }
    lj[i] = acc;
}

// log posterior and its gradient in x; with p given, then the leapfrog kick p += weps L^T grad.
__global__ void k_assemble(int64_t n, const double* __restrict__ lnl, const double* __restrict__ gth, int gs,
                           const double* __restrict__ dtdx, const double* __restrict__ lj,
                           const double* __restrict__ dlj, double* __restrict__ logp, double* __restrict__ grad,
                           double weps, double* __restrict__ p, Metric m) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool ok = isfinite(lnl[i]);
    logp[i] = ok ? lnl[i] + lj[i] : -INFINITY;
    if (grad) {
        double g[7];
        for (int j = 0; j < 7; ++j) {
            g[j] = ok ? fma(gth[i * gs + j], dtdx[i * 7 + j], dlj[i * 7 + j]) : 0.0;
            grad[i * 7 + j] = g[j];
        }
        if (p) metric_kick(m, weps, g, p + i * 7);
    }
}

__global__ void k_gauss(const double* __restrict__ x, int64_t n, pd_posterior post, double* __restrict__ logp,
                        double* __restrict__ grad) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int j = 0; j < 7; ++j) {
        const double r = x[i * 7 + j] - post.mu[j];
        acc += r * r * post.isig2[j];
        if (grad) grad[i * 7 + j] = -r * post.isig2[j];
    }
    logp[i] = -0.5 * acc;
}

// ---- HMC trajectory pieces ---------------------------------------------------------------
struct HmcArgs {
    double eps;
    Metric m;
};

// r = xi;  H0 = -logp + |r|^2 / 2;  first half kick.
__global__ void k_hmc_begin(int64_t n, HmcArgs a, const double* __restrict__ xi, const double* __restrict__ logp,
                            const double* __restrict__ grad, double* __restrict__ p, double* __restrict__ h0) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double kin = 0.0, g[7];
    for (int j = 0; j < 7; ++j) {
        const double rj = xi[i * 7 + j];
        kin = fma(rj, rj, kin);
        p[i * 7 + j] = rj;
        g[j] = grad[i * 7 + j];
    }
    metric_kick(a.m, 0.5 * a.eps, g, p + i * 7);
    h0[i] = -logp[i] + 0.5 * kin;
}

// drift: x += eps L r
__global__ void k_hmc_drift(int64_t n, HmcArgs a, double* __restrict__ x, const double* __restrict__ p) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double dx[7];
    metric_drift(a.m, a.eps, p + i * 7, dx);
    for (int j = 0; j < 7; ++j) x[i * 7 + j] += dx[j];
}

// kick: r += w eps L^T grad  (w = 1 inside the trajectory, 1/2 at its end)
__global__ void k_hmc_kick(int64_t n, HmcArgs a, double weps, double* __restrict__ p, const double* __restrict__ grad) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double g[7];
    for (int j = 0; j < 7; ++j) g[j] = grad[i * 7 + j];
    metric_kick(a.m, weps, g, p + i * 7);
}

// Metropolis-Hastings on the Hamiltonian; NaN or |dH| > 1000 (a divergence) rejects.
__global__ void k_hmc_accept(int64_t n, const double* __restrict__ u, const double* __restrict__ h0,
                             const double* __restrict__ x1, const double* __restrict__ p1,
                             const double* __restrict__ logp1, const double* __restrict__ grad1,
                             double* __restrict__ x, double* __restrict__ logp, double* __restrict__ grad,
                             int32_t* __restrict__ accepted, double* __restrict__ dh_out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double kin = 0.0;
    for (int j = 0; j < 7; ++j) kin = fma(p1[i * 7 + j], p1[i * 7 + j], kin);
    const double h1 = -logp1[i] + 0.5 * kin;
    const double dh = h1 - h0[i];
    const bool finite = isfinite(dh);
    const bool acc = finite && fabs(dh) <= 1000.0 && log(u[i]) < -dh;
    if (acc) {
        for (int j = 0; j < 7; ++j) {
            x[i * 7 + j] = x1[i * 7 + j];
            grad[i * 7 + j] = grad1[i * 7 + j];
        }
        logp[i] = logp1[i];
    }
    if (accepted) accepted[i] = acc ? 1 : ((finite && fabs(dh) <= 1000.0) ? 0 : -1);
    if (dh_out) dh_out[i] = dh;
}

// Independence Metropolis-Hastings: accept x' ~ q with prob min(1, pi(x') q(x) / (pi(x) q(x'))).
__global__ void k_imh(int64_t n, double* __restrict__ x, double* __restrict__ logp, double* __restrict__ logq,
                      double* __restrict__ grad, const double* __restrict__ xp, const double* __restrict__ logp_p,
                      const double* __restrict__ logq_p, const double* __restrict__ grad_p,
                      const double* __restrict__ u, int32_t* __restrict__ accepted) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double la = (logp_p[i] - logp[i]) + (logq[i] - logq_p[i]);
    const bool acc = isfinite(logp_p[i]) && isfinite(logq_p[i]) && (log(u[i]) < la || !isfinite(logp[i]));
    if (acc) {
        for (int j = 0; j < 7; ++j) x[i * 7 + j] = xp[i * 7 + j];
        if (grad)
            for (int j = 0; j < 7; ++j) grad[i * 7 + j] = grad_p[i * 7 + j];
        logp[i] = logp_p[i];
        logq[i] = logq_p[i];
    }
    if (accepted) accepted[i] = acc ? 1 : 0;
}

// Gaussian random-walk proposal x' = x + L xi: per coordinate (L diagonal, the step scales) or
// correlated (L lower triangular, proposal covariance L L^T).
__global__ void k_rw_propose(int64_t n, Metric m, const double* __restrict__ x, const double* __restrict__ xi,
                             double* __restrict__ xp) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double dx[7];
    metric_drift(m, 1.0, xi + i * 7, dx);
    for (int j = 0; j < 7; ++j) xp[i * 7 + j] = x[i * 7 + j] + dx[j];
}

// Metropolis accept for a symmetric proposal: accept x' with probability min(1, pi(x') / pi(x)).
// A non-finite log pi(x') rejects; a chain whose current log pi is not finite takes any finite proposal.
__global__ void k_rw_accept(int64_t n, const double* __restrict__ xp, const double* __restrict__ logp_p,
                            const double* __restrict__ u, double* __restrict__ x, double* __restrict__ logp,
                            int32_t* __restrict__ accepted) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double lpp = logp_p[i];
    const bool acc = isfinite(lpp) && (log(u[i]) < lpp - logp[i] || !isfinite(logp[i]));
    if (acc) {
        for (int j = 0; j < 7; ++j) x[i * 7 + j] = xp[i * 7 + j];
        logp[i] = lpp;
    }
    if (accepted) accepted[i] = acc ? 1 : 0;
}

inline unsigned nblk(int64_t threads, int per) { return static_cast<unsigned>((threads + per - 1) / per); }

constexpr size_t kAl = 256;
inline size_t al(size_t x) { return (x + kAl - 1) / kAl * kAl; }

// posterior workspace: theta, dtdx, dlj [n][7]; lj, lnl [n]; gth [n][7]; then loglike workspace
struct PostWs {
    double *theta, *dtdx, *dlj, *lj, *lnl, *gth;
    void* ll;
    size_t ll_bytes;
};

// parameter-row width: 11 for the network target (orientation appended), else 7
inline int row_width(const pd_posterior* post) { return post->kind == PD_TARGET_GW_NETWORK ? 11 : 7; }

size_t likelihood_ws_bytes(const pd_posterior* post, int64_t n) {
    if (post->kind == PD_TARGET_GW) return pd_workspace_bytes(PD_OP_LOGLIKE_GRAD, n, post->grid.n_bins);
    if (post->kind == PD_TARGET_GW_NETWORK) return pd_network_workspace_bytes(n, post->grid.n_bins, post->n_det);
    return 0;
}

size_t post_ws_bytes(const pd_posterior* post, int64_t n) {
    const size_t N = static_cast<size_t>(n);
    const size_t R = static_cast<size_t>(row_width(post));
    size_t off = 0;
    off = al(off + N * R * 8);
    off = al(off + N * 7 * 8);
    off = al(off + N * 7 * 8);
    off = al(off + N * 8);
    off = al(off + N * 8);
    off = al(off + N * R * 8);
    return al(off + likelihood_ws_bytes(post, n));
}

PostWs post_ws(const pd_posterior* post, int64_t n, void* base) {
    const size_t N = static_cast<size_t>(n);
    const size_t R = static_cast<size_t>(row_width(post));
    char* p = static_cast<char*>(base);
    size_t off = 0;
    PostWs w;
    w.theta = reinterpret_cast<double*>(p + off);
    off = al(off + N * R * 8);
    w.dtdx = reinterpret_cast<double*>(p + off);
    off = al(off + N * 7 * 8);
    w.dlj = reinterpret_cast<double*>(p + off);
    off = al(off + N * 7 * 8);
    w.lj = reinterpret_cast<double*>(p + off);
    off = al(off + N * 8);
    w.lnl = reinterpret_cast<double*>(p + off);
    off = al(off + N * 8);
    w.gth = reinterpret_cast<double*>(p + off);
    off = al(off + N * R * 8);
    w.ll = p + off;
    w.ll_bytes = likelihood_ws_bytes(post, n);
    return w;
}

// hmc workspace: x1, p [n][7]; h0, logp1 [n]; grad1 [n][7]; then the posterior workspace
struct HmcWs {
    double *x1, *p, *h0, *logp1, *grad1;
    void* post;
};

size_t hmc_ws_bytes(const pd_posterior* post, int64_t n) {
    const size_t N = static_cast<size_t>(n);
    size_t off = 0;
    off = al(off + N * 7 * 8);
    off = al(off + N * 7 * 8);
    off = al(off + N * 8);
    off = al(off + N * 8);
    off = al(off + N * 7 * 8);
    return off + post_ws_bytes(post, n);
}

HmcWs hmc_ws(int64_t n, void* base) {
    const size_t N = static_cast<size_t>(n);
    char* p = static_cast<char*>(base);
    size_t off = 0;
    HmcWs w;
    w.x1 = reinterpret_cast<double*>(p + off);
    off = al(off + N * 7 * 8);
    w.p = reinterpret_cast<double*>(p + off);
    off = al(off + N * 7 * 8);
    w.h0 = reinterpret_cast<double*>(p + off);
    off = al(off + N * 8);
    w.logp1 = reinterpret_cast<double*>(p + off);
    off = al(off + N * 8);
    w.grad1 = reinterpret_cast<double*>(p + off);
    off = al(off + N * 7 * 8);
    w.post = p + off;
    return w;
}

// random-walk workspace: xp [n][7]; logp_p [n]; then the posterior workspace
size_t rw_ws_bytes(const pd_posterior* post, int64_t n) {
    const size_t N = static_cast<size_t>(n);
    return al(N * 7 * 8) + al(N * 8) + post_ws_bytes(post, n);
}

}  // namespace

int posterior_check(const pd_posterior* post) {
    if (!post) return PD_EINVAL;
    if (post->kind != PD_TARGET_GW && post->kind != PD_TARGET_GAUSS && post->kind != PD_TARGET_GW_NETWORK)
        return PD_EINVAL;
    if (post->kind == PD_TARGET_GW_NETWORK) {
        if (post->n_det < 1 || post->n_det > PD_NETWORK_MAX_DETECTORS || !std::isfinite(post->gmst)) return PD_EINVAL;
        for (int d = 0; d < post->n_det; ++d)
            for (int k = 0; k < 3; ++k)
                if (!std::isfinite(post->detectors[d].vertex[k]) || !std::isfinite(post->detectors[d].xarm[k]) ||
                    !std::isfinite(post->detectors[d].yarm[k]))
                    return PD_EINVAL;
        for (int k = 0; k < 4; ++k)
            if (!std::isfinite(post->orient[k])) return PD_EINVAL;
    }
    if (post->kind != PD_TARGET_GAUSS) {
        if (!post->lambda || !post->data || !post->inv_psd) return PD_EINVAL;
        for (int j = 0; j < 7; ++j)
            if (!(post->hi[j] > post->lo[j]) || !std::isfinite(post->hi[j] - post->lo[j])) return PD_EINVAL;
        if (!(post->lo[0] > 0.0) || !(post->lo[1] > 0.0) || !(post->hi[1] <= 1.0) || !(post->lo[4] > 0.0) ||
            post->lo[2] < -1.0 || post->hi[2] > 1.0 || post->lo[3] < -1.0 || post->hi[3] > 1.0)
            return PD_EINVAL;
    } else {
        for (int j = 0; j < 7; ++j)
            if (!(post->isig2[j] > 0.0)) return PD_EINVAL;
    }
    return PD_OK;
}

// Log posterior (and gradient) at x.  Inside a leapfrog step (GW target): `drift` moves x first
// (x is then updated in place) and `kick_p` receives p += kick_weps grad afterwards, each fused into
// the neighbouring per-chain kernel.
int posterior_logp_step(const pd_posterior* post, double* x, int64_t n, double* logp, double* grad, void* ws,
                        hipStream_t s, bool tables_ready, const Drift* drift, double kick_weps, double* kick_p) {
    PostWs w = post_ws(post, n, ws);
    const int ts = row_width(post);
    if (post->kind == PD_TARGET_GW && grad) {
        // one-detector gradient pass: the drift and the coordinate map run in the record setup and
        // the log-density, gradient in x and kick in the likelihood epilogue
        XForm xf;
        xf.x = x;
        xf.p = drift ? drift->p : nullptr;
        xf.eps = drift ? drift->eps : 0.0;
        xf.m = drift ? drift->m : Metric{};
        for (int j = 0; j < 7; ++j) {
            xf.lo[j] = post->lo[j];
            xf.hi[j] = post->hi[j];
        }
        xf.dtdx = w.dtdx;
        xf.lj = w.lj;
        xf.dlj = w.dlj;
        PostTail tail{w.dtdx, w.lj, w.dlj, logp, grad, kick_p, kick_weps, drift ? drift->m : Metric{}};
        return loglike_and_grad(w.theta, n, PD_PARAM_MC_Q, &post->grid, post->lambda, post->data, post->inv_psd,
                                PD_FP64, w.lnl, w.gth, nullptr, w.ll, w.ll_bytes, s, tables_ready, true, &tail, &xf);
    }
    if (drift)
        hipLaunchKernelGGL(k_transform<true>, dim3(nblk(n, 128)), dim3(128), 0, s, x, n, *post, w.theta, w.dtdx, w.lj,
                           w.dlj, *drift, ts);
    else
        hipLaunchKernelGGL(k_transform<false>, dim3(nblk(n, 128)), dim3(128), 0, s, x, n, *post, w.theta, w.dtdx,
                           w.lj, w.dlj, Drift{}, ts);
    if (hipGetLastError() != hipSuccess) return PD_EHIP;
    int rc;
    if (post->kind == PD_TARGET_GW_NETWORK)
        rc = pd_network_loglike_and_grad(w.theta, n, PD_PARAM_MC_Q, &post->grid, post->lambda, post->n_det,
                                         post->detectors, post->gmst, post->data, post->inv_psd, w.lnl,
                                         grad ? w.gth : nullptr, nullptr, w.ll, w.ll_bytes, s);
    else
        rc = loglike_and_grad(w.theta, n, PD_PARAM_MC_Q, &post->grid, post->lambda, post->data, post->inv_psd,
                              PD_FP64, w.lnl, nullptr, nullptr, w.ll, w.ll_bytes, s, tables_ready);
    if (rc != PD_OK) return rc;
    hipLaunchKernelGGL(k_assemble, dim3(nblk(n, 128)), dim3(128), 0, s, n, w.lnl, w.gth, ts, w.dtdx, w.lj, w.dlj,
                       logp, grad, kick_weps, kick_p, drift ? drift->m : Metric{});
    return hipGetLastError() == hipSuccess ? PD_OK : PD_EHIP;
}

int posterior_logp(const pd_posterior* post, const double* x, int64_t n, double* logp, double* grad, void* ws,
                   hipStream_t s, bool tables_ready) {
    if (post->kind == PD_TARGET_GAUSS) {
        hipLaunchKernelGGL(k_gauss, dim3(nblk(n, 128)), dim3(128), 0, s, x, n, *post, logp, grad);
        return hipGetLastError() == hipSuccess ? PD_OK : PD_EHIP;
    }
    // without a drift the transform only reads x
    return posterior_logp_step(post, const_cast<double*>(x), n, logp, grad, ws, s, tables_ready, nullptr, 0.0,
                               nullptr);
}

size_t posterior_ws_bytes(const pd_posterior* post, int64_t n) { return post_ws_bytes(post, n); }
size_t hmc_workspace_bytes(const pd_posterior* post, int64_t n) { return hmc_ws_bytes(post, n); }

int hmc_step(const pd_posterior* post, int64_t n, double* x, double* logp, double* grad, const double* xi,
             const double* u, int n_leapfrog, double eps, const double* mass, const double* chol, int32_t* accepted,
             double* dh, void* ws, hipStream_t s) {
    HmcWs w = hmc_ws(n, ws);
    HmcArgs a;
    a.eps = eps;
    a.m.diag = (chol == nullptr);
    for (int j = 0; j < 7; ++j)
        for (int k = 0; k < 7; ++k)
            a.m.L[j][k] = chol ? ((k <= j) ? chol[j * 7 + k] : 0.0) : ((j == k) ? 1.0 / std::sqrt(mass[j]) : 0.0);
    const unsigned b1 = nblk(n, 128);
    hipLaunchKernelGGL(k_hmc_begin, dim3(b1), dim3(128), 0, s, n, a, xi, logp, grad, w.p, w.h0);
    if (hipMemcpyAsync(w.x1, x, static_cast<size_t>(n) * 7 * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return PD_EHIP;
    Drift dr;
    dr.eps = eps;
    dr.m = a.m;
    dr.p = w.p;
    for (int l = 0; l < n_leapfrog; ++l) {
        const double weps = (l + 1 < n_leapfrog) ? eps : 0.5 * eps;
        if (post->kind != PD_TARGET_GAUSS) {
            // drift fused into the coordinate transform, kick into the posterior assembly; the grid
            // tables depend only on the data and noise and are computed by the first step (the
            // network target recomputes them per site)
            const int rc = posterior_logp_step(post, w.x1, n, w.logp1, w.grad1, w.post, s, l > 0, &dr, weps, w.p);
            if (rc != PD_OK) return rc;
        } else {
            hipLaunchKernelGGL(k_hmc_drift, dim3(b1), dim3(128), 0, s, n, a, w.x1, w.p);
            const int rc = posterior_logp(post, w.x1, n, w.logp1, w.grad1, w.post, s);
            if (rc != PD_OK) return rc;
            hipLaunchKernelGGL(k_hmc_kick, dim3(b1), dim3(128), 0, s, n, a, weps, w.p, w.grad1);
        }
    }
    hipLaunchKernelGGL(k_hmc_accept, dim3(b1), dim3(128), 0, s, n, u, w.h0, w.x1, w.p, w.logp1, w.grad1, x, logp,
                       grad, accepted, dh);
    return hipGetLastError() == hipSuccess ? PD_OK : PD_EHIP;
}

size_t rwmh_workspace_bytes(const pd_posterior* post, int64_t n) { return rw_ws_bytes(post, n); }

int rwmh_step(const pd_posterior* post, int64_t n, double* x, double* logp, const double* xi, const double* u,
              const double* scale, const double* chol, int32_t* accepted, void* ws, hipStream_t s) {
    const size_t N = static_cast<size_t>(n);
    char* base = static_cast<char*>(ws);
    double* xp = reinterpret_cast<double*>(base);
    double* lpp = reinterpret_cast<double*>(base + al(N * 7 * 8));
    void* pws = base + al(N * 7 * 8) + al(N * 8);
    Metric m;
    m.diag = (chol == nullptr);
    for (int j = 0; j < 7; ++j)
        for (int k = 0; k < 7; ++k) m.L[j][k] = chol ? ((k <= j) ? chol[j * 7 + k] : 0.0) : ((j == k) ? scale[j] : 0.0);
    hipLaunchKernelGGL(k_rw_propose, dim3(nblk(n, 128)), dim3(128), 0, s, n, m, x, xi, xp);
    if (hipGetLastError() != hipSuccess) return PD_EHIP;
    // value only: the random walk uses no gradient
    const int rc = posterior_logp(post, xp, n, lpp, nullptr, pws, s);
    if (rc != PD_OK) return rc;
    hipLaunchKernelGGL(k_rw_accept, dim3(nblk(n, 128)), dim3(128), 0, s, n, xp, lpp, u, x, logp, accepted);
    return hipGetLastError() == hipSuccess ? PD_OK : PD_EHIP;
}

int independence_mh(int64_t n, double* x, double* logp, double* logq, double* grad, const double* xp,
                    const double* logp_p, const double* logq_p, const double* grad_p, const double* u,
                    int32_t* accepted, hipStream_t s) {
    hipLaunchKernelGGL(k_imh, dim3(nblk(n, 128)), dim3(128), 0, s, n, x, logp, logq, grad, xp, logp_p, logq_p,
                       grad_p, u, accepted);
    return hipGetLastError() == hipSuccess ? PD_OK : PD_EHIP;
}

}  // namespace pd
