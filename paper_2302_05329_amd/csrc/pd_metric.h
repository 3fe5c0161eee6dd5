// HMC metric shared by the sampler kernels and the likelihood epilogue (which applies the
// leapfrog kick of a sampler's log-density pass).
#pragma once
#include <hip/hip_runtime.h>

namespace pd {

// HMC metric.  The inverse mass matrix is M^-1 = L L^T with L lower triangular (7 x 7); the chains
// carry the whitened momentum r = L^T p, so that r ~ N(0, I), the drift is x += eps L r, the kick is
// r += w eps L^T grad log pi and the kinetic energy is |r|^2 / 2.  A diagonal mass m_j is the case
// L = diag(1 / sqrt(m_j)).
struct Metric {
    double L[7][7];
    bool diag;
};

__device__ __forceinline__ void metric_drift(const Metric& m, double eps, const double* __restrict__ r, double out[7]) {
    for (int j = 0; j < 7; ++j) {
        double acc = 0.0;
        if (m.diag) {
            acc = m.L[j][j] * r[j];
        } else {
            for (int k = 0; k <= j; ++k) acc = fma(m.L[j][k], r[k], acc);
        }
        out[j] = eps * acc;
    }
}

// r += weps L^T g
__device__ __forceinline__ void metric_kick(const Metric& m, double weps, const double g[7], double* __restrict__ r) {
    for (int j = 0; j < 7; ++j) {
        double acc = 0.0;
        if (m.diag) {
            acc = m.L[j][j] * g[j];
        } else {
            for (int k = j; k < 7; ++k) acc = fma(m.L[k][j], g[k], acc);
        }
        r[j] = fma(weps, acc, r[j]);
    }
}

// Per-point tail of a sampler's log-density pass, fused into the likelihood-gradient epilogue:
// logp = ln L + lj, grad = d ln L / d theta * dtdx + dlj (the coordinate map is elementwise), and,
// with p set, the leapfrog kick p += weps L^T grad.  A point whose ln L is not finite gets
// logp = -inf and a zero gradient (no kick).
struct PostTail {
    const double* dtdx;
    const double* lj;
    const double* dlj;
    double* logp;
    double* grad;
    double* p;
    double weps;
    Metric m;
};

// The sampler's coordinate map applied by the record setup of a log-density pass: with p set,
// first the leapfrog drift x += eps L p (x updated in place); then
// theta_j = lo_j + (hi_j - lo_j) sigmoid(x_j), written to the pass's theta rows, with d theta / d x,
// the log-Jacobian sum_j log(d theta_j / d x_j) and its derivative.
struct XForm {
    double* x;
    const double* p;
    double eps;
    Metric m;
    double lo[7], hi[7];
    double* dtdx;
    double* lj;
    double* dlj;
};

__device__ __forceinline__ double xform_sigmoid(double x) {
    return (x >= 0.0) ? 1.0 / (1.0 + exp(-x)) : exp(x) / (1.0 + exp(x));
}

// Point i of the map; theta_row receives the 7 parameters.
__device__ __forceinline__ void xform_point(const XForm& f, int64_t i, double theta_row[7]) {
    double dx[7];
    if (f.p) metric_drift(f.m, f.eps, f.p + i * 7, dx);
    double acc = 0.0;
    for (int j = 0; j < 7; ++j) {
        double xv = f.x[i * 7 + j];
        if (f.p) {
            xv += dx[j];
            f.x[i * 7 + j] = xv;
        }
        const double s = xform_sigmoid(xv);
        const double w = f.hi[j] - f.lo[j];
        theta_row[j] = f.lo[j] + w * s;
        f.dtdx[i * 7 + j] = w * s * (1.0 - s);
        // log(w s (1-s)) = log w - softplus(-x) - softplus(x)
        const double ax = fabs(xv);
        acc += log(w) - ax - 2.0 * log1p(exp(-ax));
        f.dlj[i * 7 + j] = 1.0 - 2.0 * s;
    }
    f.lj[i] = acc;
}

}  // namespace pd
