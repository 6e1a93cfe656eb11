// Primal-dual interior-point kernels for P(N) with bounds on the inputs,
// wlo_t <= w_t <= whi_t: the constrained MHE problem whose Newton steps the
// paper's solver computes (Sec. 3: each IP iteration solves an equality
// constrained problem of the form P(N)).
//
// With slacks s_l = w - wlo, s_u = whi - w and bound multipliers m_l, m_u >= 0
// the KKT residuals at the current point are
//   r_x = Qx x_t + Qxw w_t + lx_t - lam_t + A' lam_{t+1}      (r_x,N = QxN x_N + lN - lam_N)
//   r_w = Qxw' x_t + Qw w_t + lw_t + B' lam_{t+1} - m_l + m_u
//   r_l = A x_t + B w_t + a_t - x_{t+1},     r_0 = x_0 - xbar_0
//   r_cl = s_l m_l - sigma mu (+ ds_l dm_l of the affine step),  r_cu likewise.
// Eliminating the multiplier steps (dm_l = -(r_cl + m_l dw) / s_l,
// dm_u = -(r_cu - m_u dw) / s_u) leaves the Newton system of a problem of the
// form P(N) in (dx, dw, dlam) with Q_w + Sigma, Sigma = m_l / s_l + m_u / s_u,
// and right-hand side lx' = r_x, lw' = r_w + r_cl / s_l - r_cu / s_u,
// a' = r_l, xbar_0' = -r_0, lN' = r_x,N: its solution is the step.  The
// factorization of Q_w + Sigma is shared by the predictor (sigma = 0) and the
// corrector (Mehrotra) solves.
//
// One wavefront per stage (block N: terminal and initial rows); per-stage
// partial results are reduced per instance in a fixed order by k_ip_reduce.
#include <hip/hip_runtime.h>

#include "rs.h"
#include "rs_device.hpp"

namespace rs {
namespace ip {

constexpr int WT = 64;
constexpr int MAXN = 64;
constexpr double BIG = 1e300;     // |bound| beyond this: no bound on that side

// Partial results per stage: PX max|r_x|, PW max|r_w|, PL max|r_l| (and r_0),
// PC sum of s m, PN bounded sides, PAP / PAD largest primal / dual step in
// (0, 1], PMU sum of (s + a ds)(m + a dm) at the affine step.
enum { PX = 0, PW = 1, PL = 2, PC = 3, PN = 4, PAP = 5, PAD = 6, PMU = 7, NP = 8 };

struct View {
    rs_ip a;
    __device__ const double *blk(const double *b, int64_t s, int t) const { return b + (int64_t)t * s; }
};

__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wmin(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Complementarity residuals of component j of stage t for the given phase.
struct Comp {
    bool lo, hi;
    double sl, su, rcl, rcu;
};
__device__ __forceinline__ Comp comp(const rs_ip &a, int t, int j, double w, int phase, double sigma_mu) {
    const int64_t e = (int64_t)t * a.nu + j;
    const double wl = a.wlo[(int64_t)t * a.swlo + j], wh = a.whi[(int64_t)t * a.swhi + j];
    Comp c;
    c.lo = wl > -BIG;
    c.hi = wh < BIG;
    c.sl = c.lo ? w - wl : 1.0;
    c.su = c.hi ? wh - w : 1.0;
    const double ml = a.ml[e], mu = a.mu[e];
    c.rcl = c.lo ? c.sl * ml : 0.0;
    c.rcu = c.hi ? c.su * mu : 0.0;
    if (phase == 1) {
        const double dw = a.dw_aff[e];
        if (c.lo) c.rcl += dw * a.dml[e] - sigma_mu;
        if (c.hi) c.rcu += -dw * a.dmu[e] - sigma_mu;
    }
    return c;
}

// Residuals and the Newton system's data.  phase 0 (predictor) also writes
// Q_w + Sigma and the residual norms; phase 1 (corrector) only the input
// linear term.
__global__ void __launch_bounds__(WT) k_ip_newton(rs_ip a, int phase, double sigma_mu) {
    __shared__ double sx[MAXN], sw[MAXN], sl0[MAXN], sl1[MAXN], sxn[MAXN];
    const int n = a.nx, m = a.nu, N = a.N, t = blockIdx.x, l = threadIdx.x;
    const rs_problem &p = a.prob, &q = a.newton;
    double *part = a.part + (int64_t)t * NP;
    if (t == N) {
        // terminal row and initial condition
        for (int i = l; i < n; i += WT) {
            sx[i] = p.x[(int64_t)N * n + i];
            sl0[i] = p.lam[(int64_t)N * n + i];
        }
        wsync();
        double rx = 0.0, r0 = 0.0;
        for (int i = l; i < n; i += WT) {
            double s = (p.lN ? p.lN[i] : 0.0) - sl0[i];
            for (int j = 0; j < n; ++j) s += p.QxN[i * n + j] * sx[j];
            const double d0 = p.x0[i] - p.x[i];           // xbar_0 - x_0
            if (phase == 0) {
                const_cast<double *>(q.lN)[i] = s;
                const_cast<double *>(q.x0)[i] = d0;
            }
            rx = fmax(rx, fabs(s));
            r0 = fmax(r0, fabs(d0));
        }
        rx = wmax(rx);
        r0 = wmax(r0);
        if (l == 0 && phase == 0) {
            part[PX] = rx;
            part[PW] = 0.0;
            part[PL] = r0;
            part[PC] = 0.0;
            part[PN] = 0.0;
        }
        return;
    }
    for (int i = l; i < n; i += WT) {
        sx[i] = p.x[(int64_t)t * n + i];
        sxn[i] = p.x[(int64_t)(t + 1) * n + i];
        sl0[i] = p.lam[(int64_t)t * n + i];
        sl1[i] = p.lam[(int64_t)(t + 1) * n + i];
    }
    for (int j = l; j < m; j += WT) sw[j] = p.w[(int64_t)t * m + j];
    wsync();
    const double *Qx = p.Qx + (int64_t)t * p.sQx, *Qw = p.Qw + (int64_t)t * p.sQw;
    const double *Qxw = p.Qxw ? p.Qxw + (int64_t)t * p.sQxw : nullptr;
    const double *A = p.A + (int64_t)t * p.sA, *B = p.B + (int64_t)t * p.sB;
    double mrx = 0.0, mrw = 0.0, mrl = 0.0, csum = 0.0, nb = 0.0;
    for (int i = l; i < n; i += WT) {
        double rx = (p.lx ? p.lx[(int64_t)t * p.slx + i] : 0.0) - sl0[i];
        double rl = (p.a ? p.a[(int64_t)t * p.sa + i] : 0.0) - sxn[i];
        for (int j = 0; j < n; ++j) {
            rx += Qx[i * n + j] * sx[j] + A[j * n + i] * sl1[j];
            rl += A[i * n + j] * sx[j];
        }
        for (int k = 0; k < m; ++k) {
            if (Qxw) rx += Qxw[i * m + k] * sw[k];
            rl += B[i * m + k] * sw[k];
        }
        const_cast<double *>(q.lx)[(int64_t)t * q.slx + i] = rx;
        if (phase == 0) const_cast<double *>(q.a)[(int64_t)t * q.sa + i] = rl;
        mrx = fmax(mrx, fabs(rx));
        mrl = fmax(mrl, fabs(rl));
    }
    double *Qm = const_cast<double *>(q.Qw) + (int64_t)t * q.sQw;
    for (int j = l; j < m; j += WT) {
        const int64_t e = (int64_t)t * m + j;
        double rw = (p.lw ? p.lw[(int64_t)t * p.slw + j] : 0.0) - a.ml[e] + a.mu[e];
        for (int i = 0; i < n; ++i) {
            if (Qxw) rw += Qxw[i * m + j] * sx[i];
            rw += B[i * m + j] * sl1[i];
        }
        for (int k = 0; k < m; ++k) rw += Qw[j * m + k] * sw[k];
        const Comp c = comp(a, t, j, sw[j], phase, sigma_mu);
        double sig = 0.0, rt = rw;
        if (c.lo) {
            sig += a.ml[e] / c.sl;
            rt += c.rcl / c.sl;
        }
        if (c.hi) {
            sig += a.mu[e] / c.su;
            rt -= c.rcu / c.su;
        }
        const_cast<double *>(q.lw)[(int64_t)t * q.slw + j] = rt;
        if (phase == 0) {
            for (int k = 0; k < m; ++k) Qm[j * m + k] = Qw[j * m + k] + (k == j ? sig : 0.0);
            mrw = fmax(mrw, fabs(rw));
            csum += c.rcl + c.rcu;
            nb += (c.lo ? 1.0 : 0.0) + (c.hi ? 1.0 : 0.0);
        }
    }
    if (phase == 0) {
        mrx = wmax(mrx);
        mrw = wmax(mrw);
        mrl = wmax(mrl);
        csum = wsum(csum);
        nb = wsum(nb);
        if (l == 0) {
            part[PX] = mrx;
            part[PW] = mrw;
            part[PL] = mrl;
            part[PC] = csum;
            part[PN] = nb;
            const_cast<double *>(q.c)[(int64_t)t * q.sc] = 0.0;
        }
    }
}

// After the solve of `phase`: multiplier steps and the largest feasible step
// lengths.  Phase 0 keeps the affine step (dw_aff, dml, dmu); phase 1
// overwrites dml, dmu with the corrector's multiplier steps.
__global__ void __launch_bounds__(WT) k_ip_step(rs_ip a, int phase, double sigma_mu) {
    const int m = a.nu, t = blockIdx.x, l = threadIdx.x;
    double ap = 1.0, ad = 1.0;
    for (int j = l; j < m; j += WT) {
        const int64_t e = (int64_t)t * m + j;
        const double w = a.prob.w[e], dw = a.newton.w[e];
        const Comp c = comp(a, t, j, w, phase, sigma_mu);
        const double ml = a.ml[e], mu = a.mu[e];
        const double dml = c.lo ? -(c.rcl + ml * dw) / c.sl : 0.0;
        const double dmu = c.hi ? -(c.rcu - mu * dw) / c.su : 0.0;
        if (c.lo && dw < 0.0) ap = fmin(ap, -c.sl / dw);
        if (c.hi && dw > 0.0) ap = fmin(ap, c.su / dw);
        if (dml < 0.0) ad = fmin(ad, -ml / dml);
        if (dmu < 0.0) ad = fmin(ad, -mu / dmu);
        a.dml[e] = dml;
        a.dmu[e] = dmu;
        if (phase == 0) a.dw_aff[e] = dw;
    }
    ap = wmin(ap);
    ad = wmin(ad);
    if (l == 0) {
        a.part[(int64_t)t * NP + PAP] = ap;
        a.part[(int64_t)t * NP + PAD] = ad;
    }
}

// Complementarity at the affine step (Mehrotra's centring estimate).
__global__ void __launch_bounds__(WT) k_ip_mu(rs_ip a, double ap, double ad) {
    const int m = a.nu, t = blockIdx.x, l = threadIdx.x;
    double s = 0.0;
    for (int j = l; j < m; j += WT) {
        const int64_t e = (int64_t)t * m + j;
        const double w = a.prob.w[e], dw = a.dw_aff[e];
        const Comp c = comp(a, t, j, w, 0, 0.0);
        if (c.lo) s += (c.sl + ap * dw) * (a.ml[e] + ad * a.dml[e]);
        if (c.hi) s += (c.su - ap * dw) * (a.mu[e] + ad * a.dmu[e]);
    }
    s = wsum(s);
    if (l == 0) a.part[(int64_t)t * NP + PMU] = s;
}

// Iterate update with the corrector's step.
__global__ void __launch_bounds__(WT) k_ip_update(rs_ip a, double ap, double ad) {
    const int n = a.nx, m = a.nu, N = a.N, t = blockIdx.x, l = threadIdx.x;
    const rs_problem &p = a.prob, &q = a.newton;
    for (int i = l; i < n; i += WT) {
        const int64_t e = (int64_t)t * n + i;
        p.x[e] += ap * q.x[e];
        p.lam[e] += ad * q.lam[e];
    }
    if (t == N) return;
    for (int j = l; j < m; j += WT) {
        const int64_t e = (int64_t)t * m + j;
        p.w[e] += ap * q.w[e];
        a.ml[e] += ad * a.dml[e];
        a.mu[e] += ad * a.dmu[e];
    }
}

// Fixed-order reduction of the per-stage partials into stats[0 .. NP).
__global__ void __launch_bounds__(WT) k_ip_reduce(rs_ip a, int nstage, int first, int count) {
    const int l = threadIdx.x;
    for (int k = first; k < first + count; ++k) {
        const bool mx = k == PX || k == PW || k == PL, mn = k == PAP || k == PAD;
        double v = mx ? 0.0 : mn ? 1.0 : 0.0;
        for (int t = l; t < nstage; t += WT) {
            const double x = a.part[(int64_t)t * NP + k];
            v = mx ? fmax(v, x) : mn ? fmin(v, x) : v + x;
        }
        v = mx ? wmax(v) : mn ? wmin(v) : wsum(v);
        if (l == 0) a.stats[k] = v;
    }
}

bool valid(const rs_ip &a) {
    return a.nx >= 1 && a.nu >= 1 && a.N >= 1 && a.nx <= MAXN && a.nu <= MAXN && a.prob.nx == a.nx &&
           a.prob.nu == a.nu && a.prob.N == a.N && a.newton.nx == a.nx && a.newton.nu == a.nu && a.newton.N == a.N &&
           a.wlo && a.whi && a.ml && a.mu && a.dw_aff && a.dml && a.dmu && a.part && a.stats && a.prob.x && a.prob.w &&
           a.prob.lam && a.newton.x && a.newton.w && a.newton.lam && a.newton.Qw && a.newton.lx && a.newton.lw &&
           a.newton.a && a.newton.c && a.newton.lN && a.newton.x0;
}

}  // namespace ip
}  // namespace rs

using namespace rs::ip;

extern "C" rs_status rs_ip_newton(const rs_ip *a, int32_t phase, double sigma_mu, void *stream) {
    if (!a || !valid(*a) || (phase != 0 && phase != 1)) return RS_ERR_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_ip_newton, dim3(a->N + 1), dim3(WT), 0, st, *a, (int)phase, sigma_mu);
    if (hipGetLastError() != hipSuccess) return RS_ERR_HIP;
    if (phase == 0) hipLaunchKernelGGL(k_ip_reduce, dim3(1), dim3(WT), 0, st, *a, a->N + 1, (int)PX, 5);
    return hipGetLastError() == hipSuccess ? RS_OK : RS_ERR_HIP;
}

extern "C" rs_status rs_ip_step(const rs_ip *a, int32_t phase, double sigma_mu, void *stream) {
    if (!a || !valid(*a) || (phase != 0 && phase != 1)) return RS_ERR_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_ip_step, dim3(a->N), dim3(WT), 0, st, *a, (int)phase, sigma_mu);
    if (hipGetLastError() != hipSuccess) return RS_ERR_HIP;
    hipLaunchKernelGGL(k_ip_reduce, dim3(1), dim3(WT), 0, st, *a, a->N, (int)PAP, 2);
    return hipGetLastError() == hipSuccess ? RS_OK : RS_ERR_HIP;
}

extern "C" rs_status rs_ip_mu(const rs_ip *a, double alpha_p, double alpha_d, void *stream) {
    if (!a || !valid(*a)) return RS_ERR_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_ip_mu, dim3(a->N), dim3(WT), 0, st, *a, alpha_p, alpha_d);
    if (hipGetLastError() != hipSuccess) return RS_ERR_HIP;
    hipLaunchKernelGGL(k_ip_reduce, dim3(1), dim3(WT), 0, st, *a, a->N, (int)PMU, 1);
    return hipGetLastError() == hipSuccess ? RS_OK : RS_ERR_HIP;
}

extern "C" rs_status rs_ip_update(const rs_ip *a, double alpha_p, double alpha_d, void *stream) {
    if (!a || !valid(*a)) return RS_ERR_ARG;
    hipLaunchKernelGGL(k_ip_update, dim3(a->N + 1), dim3(WT), 0, reinterpret_cast<hipStream_t>(stream), *a,
                       alpha_p, alpha_d);
    return hipGetLastError() == hipSuccess ? RS_OK : RS_ERR_HIP;
}
