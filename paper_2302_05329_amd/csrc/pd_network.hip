// Detector-network likelihood (the two-detector injection of Sec. 3.3, the network Fisher setups
// of Sec. 3.2): per-site antenna response, arrival delay and the network ln L with its gradient
// over 11 parameters (the 7 of the single-detector model, then inclination, polarisation, right
// ascension and declination).
//
// For the dominant (2,2) mode the strain a site records is the face-on, optimally oriented model
// strain h0 times c = F+ (1 + cos^2 iota)/2 - i Fx cos iota, delayed by dt = -(r . n)/c_light.
// Because h0 depends on the distance as 1/D, on tc through exp(-2 pi i f tc) and on phic through
// exp(2 i phic), that strain is exactly the single-detector model at the effective parameters
//   D_d = D / |c|,   tc_d = tc + dt,   phic_d = phic + arg(c) / 2,
// so each site is one fused likelihood pass of the single-detector kernels at its effective
// parameters and its own data and noise.  This file holds the two per-point kernels around those
// passes: the effective parameters with their derivatives, and the sum over sites with the chain
// rule to the 11 parameters.  The network Fisher matrix (Eq. 8 summed over sites) is built the same
// way from one single-site Fisher pass per site: F = sum over sites of J^T F_d J, with J the
// Jacobian of the site's effective row.
//
// Frame: Earth-fixed; source direction n = (cos d cos l, cos d sin l, sin d), l = alpha - gmst;
// wave axes a = (sin l, -cos l, 0), b = n x a = (sin d cos l, sin d sin l, -cos d), and
// X = cos psi a + sin psi b, Y = -sin psi a + cos psi b; e+ = XX - YY, ex = XY + YX; the site
// tensor is D = (x x - y y)/2.  With F+0 = a.D.a - b.D.b and Fx0 = 2 a.D.b (psi = 0),
// F+ = cos 2psi F+0 + sin 2psi Fx0 and Fx = -sin 2psi F+0 + cos 2psi Fx0.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/phenomd.h"
#include "pd_launch.h"

namespace pd {

namespace {

constexpr double kCLight = 299792458.0;

__device__ __forceinline__ double dot3(const double* u, const double* v) {
    return u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
}

// u . D . v with D = (x x^T - y y^T) / 2
__device__ __forceinline__ double dten(const NetSite& st, const double* u, const double* v) {
    return 0.5 * (dot3(u, st.xarm) * dot3(v, st.xarm) - dot3(u, st.yarm) * dot3(v, st.yarm));
}

// Per point: for each site the effective 7-parameter row and the derivatives of its entries
// 4 (D or ln D), 5 (tc) and 6 (phic) w.r.t. (iota, psi, alpha, delta), plus d row4 / d theta4.
// jac layout per (site, point): [0] d row4/d theta4, [1 + 4k + m] d row(4+k) / d x_m.
__global__ void __launch_bounds__(128) k_net_setup(const double* __restrict__ theta, int64_t n, int param,
                                                   NetArgs na, double* __restrict__ eff,
                                                   double* __restrict__ jac) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* th = theta + i * kNetParams;
    const double iota = th[7], psi = th[8], alpha = th[9], delta = th[10];
    const double lam = alpha - na.gmst;
    const double cd = cos(delta), sd = sin(delta), cl = cos(lam), sl = sin(lam);
    const double nv[3] = {cd * cl, cd * sl, sd};
    const double nl[3] = {-cd * sl, cd * cl, 0.0};       // d n / d alpha
    const double nd[3] = {-sd * cl, -sd * sl, cd};       // d n / d delta
    const double av[3] = {sl, -cl, 0.0};
    const double al[3] = {cl, sl, 0.0};                  // d a / d alpha  (d a / d delta = 0)
    const double bv[3] = {sd * cl, sd * sl, -cd};
    const double bl[3] = {-sd * sl, sd * cl, 0.0};       // d b / d alpha
    const double* bd = nv;                               // d b / d delta = n
    const double c2p = cos(2.0 * psi), s2p = sin(2.0 * psi);
    const double ci = cos(iota), si = sin(iota);
    const double kp = 0.5 * (1.0 + ci * ci);
    for (int d = 0; d < na.n_det; ++d) {
        const NetSite& st = na.site[d];
        const double fp0 = dten(st, av, av) - dten(st, bv, bv);
        const double fx0 = 2.0 * dten(st, av, bv);
        const double fp0_a = 2.0 * (dten(st, al, av) - dten(st, bl, bv));
        const double fx0_a = 2.0 * (dten(st, al, bv) + dten(st, av, bl));
        const double fp0_d = -2.0 * dten(st, bd, bv);
        const double fx0_d = 2.0 * dten(st, av, bd);
        const double fp = c2p * fp0 + s2p * fx0, fx = -s2p * fp0 + c2p * fx0;
        // derivatives of (F+, Fx) w.r.t. (psi, alpha, delta)
        const double dfp[3] = {2.0 * fx, c2p * fp0_a + s2p * fx0_a, c2p * fp0_d + s2p * fx0_d};
        const double dfx[3] = {-2.0 * fp, -s2p * fp0_a + c2p * fx0_a, -s2p * fp0_d + c2p * fx0_d};
        const double cr = fp * kp, cim = -fx * ci;
        // derivatives of (cr, ci) w.r.t. (iota, psi, alpha, delta)
        double dcr[4], dci[4];
        dcr[0] = -fp * ci * si;
        dci[0] = fx * si;
        for (int m = 0; m < 3; ++m) {
            dcr[m + 1] = dfp[m] * kp;
            dci[m + 1] = -dfx[m] * ci;
        }
        const double c2 = cr * cr + cim * cim;
        double* e = eff + (static_cast<int64_t>(d) * n + i) * 7;
        double* J = jac + (static_cast<int64_t>(d) * n + i) * kNetJac;
        for (int k = 0; k < 4; ++k) e[k] = th[k];
        if (c2 == 0.0) {
            // a site with no response to this source records no signal: it contributes nothing to
            // ln L, its gradient or the Fisher matrix (J[0] = 0 marks it; its pass runs on the
            // unshifted row and is ignored)
            for (int k = 4; k < 7; ++k) e[k] = th[k];
            for (int k = 0; k < kNetJac; ++k) J[k] = 0.0;
            continue;
        }
        const double ic2 = 1.0 / c2;
        const double lnc = 0.5 * log(c2);
        const double argc = atan2(cim, cr);
        const double dt = -dot3(st.vertex, nv) / kCLight;
        const double dt_a = -dot3(st.vertex, nl) / kCLight, dt_d = -dot3(st.vertex, nd) / kCLight;
        const bool lnd = (param == PD_PARAM_LNMC_ETA_LND);
        const double row4 = lnd ? th[4] - lnc : th[4] * exp(-lnc);
        e[4] = row4;
        e[5] = th[5] + dt;
        e[6] = th[6] + 0.5 * argc;
        J[0] = lnd ? 1.0 : exp(-lnc);
        for (int m = 0; m < 4; ++m) {
            const double dlnc = (cr * dcr[m] + cim * dci[m]) * ic2;
            const double darg = (cr * dci[m] - cim * dcr[m]) * ic2;
            J[1 + m] = lnd ? -dlnc : -row4 * dlnc;
            J[5 + m] = (m == 2) ? dt_a : ((m == 3) ? dt_d : 0.0);
            J[9 + m] = 0.5 * darg;
        }
    }
}

// Per point: ln L = sum over sites; the gradient by the chain rule through the effective rows.
// A point is invalid (status PD_EDOMAIN, NaN outputs) if any site's row is.
__global__ void __launch_bounds__(128) k_net_combine(int64_t n, int n_det, const double* __restrict__ lnl_d,
                                                     const double* __restrict__ grad_d,
                                                     const int32_t* __restrict__ status_d,
                                                     const double* __restrict__ jac, double* __restrict__ lnl,
                                                     double* __restrict__ grad, int32_t* __restrict__ status) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    double g[kNetParams];
    for (int p = 0; p < kNetParams; ++p) g[p] = 0.0;
    bool ok = true;
    for (int d = 0; d < n_det; ++d) {
        const int64_t r = static_cast<int64_t>(d) * n + i;
        const double* J = jac + r * kNetJac;
        if (J[0] == 0.0) {
            // a silent site: only the validity of the source itself (its status) matters
            ok = ok && status_d[r] == 0;
            continue;
        }
        ok = ok && status_d[r] == 0;
        s += lnl_d[r];
        if (grad) {
            const double* gd = grad_d + r * 7;
            for (int p = 0; p < 4; ++p) g[p] += gd[p];
            g[4] += gd[4] * J[0];
            g[5] += gd[5];
            g[6] += gd[6];
            for (int m = 0; m < 4; ++m) g[7 + m] += gd[4] * J[1 + m] + gd[5] * J[5 + m] + gd[6] * J[9 + m];
        }
    }
    const double nan = __builtin_nan("");
    lnl[i] = ok ? s : nan;
    if (grad)
        for (int p = 0; p < kNetParams; ++p) grad[i * kNetParams + p] = ok ? g[p] : nan;
    if (status) status[i] = ok ? PD_OK : PD_EDOMAIN;
}

// Nonzero entries of column p of the 7 x 11 Jacobian d(effective row) / d(theta) of one site:
// the identity on the first 7 columns (with d row4 / d theta4 at (4, 4)), rows 4-6 on the last 4.
__device__ __forceinline__ int jac_col(int p, const double* __restrict__ J, int* rows, double* vals) {
    if (p < 7) {
        rows[0] = p;
        vals[0] = (p == 4) ? J[0] : 1.0;
        return 1;
    }
    const int m = p - 7;
    for (int k = 0; k < 3; ++k) {
        rows[k] = 4 + k;
        vals[k] = J[1 + 4 * k + m];
    }
    return 3;
}

// Network Fisher matrix: F = sum over sites of J^T F_d J, one thread per (point, entry).
__global__ void __launch_bounds__(128) k_net_fisher_combine(int64_t n, int n_det, const double* __restrict__ F_d,
                                                            const int32_t* __restrict__ status_d,
                                                            const double* __restrict__ jac, double* __restrict__ F,
                                                            int32_t* __restrict__ status) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n * kNetParams * kNetParams) return;
    const int64_t i = t / (kNetParams * kNetParams);
    const int e = static_cast<int>(t % (kNetParams * kNetParams));
    // both (p, q) and (q, p) are summed in the order of (min, max): the result is exactly symmetric
    const int p = min(e / kNetParams, e % kNetParams), q = max(e / kNetParams, e % kNetParams);
    double s = 0.0;
    bool ok = true;
    for (int d = 0; d < n_det; ++d) {
        const int64_t r = static_cast<int64_t>(d) * n + i;
        ok = ok && status_d[r] == 0;
        const double* J = jac + r * kNetJac;
        if (J[0] == 0.0) continue;  // a silent site adds nothing
        const double* Fd = F_d + r * 49;
        int ra[3], rb[3];
        double va[3], vb[3];
        const int na = jac_col(p, J, ra, va), nb = jac_col(q, J, rb, vb);
        for (int a = 0; a < na; ++a)
            for (int b = 0; b < nb; ++b) s += va[a] * Fd[ra[a] * 7 + rb[b]] * vb[b];
    }
    F[i * kNetParams * kNetParams + e] = ok ? s : __builtin_nan("");
    if (status && e == 0) status[i] = ok ? PD_OK : PD_EDOMAIN;
}

inline unsigned nblk(int64_t threads, int per) { return static_cast<unsigned>((threads + per - 1) / per); }

}  // namespace

hipError_t launch_net_setup(const double* theta, int64_t n, int param, const NetArgs& na, double* eff, double* jac,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_net_setup, dim3(nblk(n, 128)), dim3(128), 0, s, theta, n, param, na, eff, jac);
    return hipGetLastError();
}

hipError_t launch_net_combine(int64_t n, int n_det, const double* lnl_d, const double* grad_d, const int32_t* status_d,
                              const double* jac, double* lnl, double* grad, int32_t* status, hipStream_t s) {
    hipLaunchKernelGGL(k_net_combine, dim3(nblk(n, 128)), dim3(128), 0, s, n, n_det, lnl_d, grad_d, status_d, jac, lnl,
                       grad, status);
    return hipGetLastError();
}

hipError_t launch_net_fisher_combine(int64_t n, int n_det, const double* F_d, const int32_t* status_d, const double* jac,
                                     double* F, int32_t* status, hipStream_t s) {
    hipLaunchKernelGGL(k_net_fisher_combine, dim3(nblk(n * kNetParams * kNetParams, 128)), dim3(128), 0, s, n, n_det,
                       F_d, status_d, jac, F, status);
    return hipGetLastError();
}

}  // namespace pd
