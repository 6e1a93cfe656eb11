// MHE front-end: the moving-horizon estimation problem of Sec. 2 (eq.
// org_mhe) written as the UFTOC problem P(N) on the device.
//
// A state x_{-1} = xtil_0 and a noise w_{-1} = x_0 - xtil_0 are prepended and
// time is shifted by t = k + 1, N = N_mhe + 2 (Sec. 2).  UFTOC stage 0 holds the
// arrival cost: Q_x = 0, Q_xw = 0, Q_w = Ptil_0^{-1}, A = I, B = I, a = 0,
// l = 0, c = 0; the terminal cost is zero and xbar_0 = xtil_0.  Stage
// t = k + 1 carries sample k: with [[W, S], [S', V]] the inverse of the joint
// covariance [[Q_w, Q_wv], [Q_wv', Q_v]] of (w_k, v_k) and ytil = y - d - vtil,
// eliminating v_k = y_k - C_k x_k - d_k from the stage cost gives
//   Q_x = C'VC,  Q_xw = -C'S',  Q_w = W,
//   l_x = C'(S' wtil - V ytil),  l_w = S ytil - W wtil,
// and A, B, a are the sample's.  The stage-0 noise has n_x components and the
// samples' n_w; P(N) has one input dimension, so every stage's input is
// padded to n_u = max(n_x, n_w) with inputs that act on nothing (zero columns
// of B and Q_xw, an identity block of Q_w, zero l_w): they are decoupled and
// strictly convex, so they are zero at the optimum.
//
// One wavefront per UFTOC stage: the (n_w + n_y) x (n_w + n_y) covariance is
// inverted by Gauss-Jordan elimination in LDS (lane r owns row r; the
// covariance is symmetric positive definite, so no pivoting is needed), then
// the products above are formed with lanes over output elements.
#include <hip/hip_runtime.h>

#include "rs.h"
#include "rs_device.hpp"

namespace rs {
namespace mhe {

constexpr int WT = 64;
constexpr int MAXD = 48;        // n_w + n_y and n_x (the covariances and their inverses in LDS)

__device__ __forceinline__ void wfence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// [M | I] -> [I | M^{-1}] for the d x d SPD matrix in the left half of the
// d x 2d row-major LDS array G.  Returns false (wave-uniform) if a pivot is
// not positive and finite.
__device__ bool gauss_jordan(double *G, int d) {
    const int r = threadIdx.x, w = 2 * d;
    bool ok = true;
    for (int p = 0; p < d; ++p) {
        const double piv = G[p * w + p];
        if (!(piv > 0.0) || !(piv < 1e300)) ok = false;
        const double inv = ok ? 1.0 / piv : 1.0;
        const double f = (r < d && r != p) ? G[r * w + p] * inv : 0.0;
        wfence();
        if (r < d && r != p)
            for (int c = 0; c < w; ++c) G[r * w + c] -= f * G[p * w + c];
        wfence();
        if (r == p)
            for (int c = 0; c < w; ++c) G[p * w + c] *= inv;
        wfence();
    }
    return ok;
}

__device__ __forceinline__ double at(const double *base, int64_t stride, int k, int e) {
    return base ? base[(int64_t)k * stride + e] : 0.0;
}

__global__ void __launch_bounds__(WT) k_mhe_convert(rs_mhe m, rs_problem o, int32_t *info) {
    extern __shared__ double lds[];
    const int nx = m.nx, ny = m.ny, nw = m.nw > 0 ? m.nw : m.nx, nu = nx > nw ? nx : nw, d = nw + ny;
    const int l = threadIdx.x, t = blockIdx.x;
    double *G = lds;                       // d x 2d (stage 0: nx x 2nx)
    const int gsz = 2 * (d > nx ? d : nx) * (d > nx ? d : nx);
    double *T = G + gsz;                   // V C (ny x nx)
    double *yt = T + ny * nx;              // ytil (ny)
    double *wt = yt + ny;                  // wtil (nw)
    double *u = wt + nw;                   // S' wtil - V ytil (ny)
    double *Qx = const_cast<double *>(o.Qx) + (int64_t)t * o.sQx;
    double *Qw = const_cast<double *>(o.Qw) + (int64_t)t * o.sQw;
    double *Qxw = o.Qxw ? const_cast<double *>(o.Qxw) + (int64_t)t * o.sQxw : nullptr;
    double *A = const_cast<double *>(o.A) + (int64_t)t * o.sA;
    double *B = const_cast<double *>(o.B) + (int64_t)t * o.sB;
    double *a = const_cast<double *>(o.a) + (int64_t)t * o.sa;
    double *lx = const_cast<double *>(o.lx) + (int64_t)t * o.slx;
    double *lw = const_cast<double *>(o.lw) + (int64_t)t * o.slw;
    double *c = const_cast<double *>(o.c) + (int64_t)t * o.sc;
    if (t == 0) {
        // arrival cost on w_{-1} = x_0 - xtil_0 (the first n_x inputs); zero terminal cost
        const int w2 = 2 * nx;
        for (int e = l; e < nx * nx; e += WT) {
            const int i = e / nx, j = e % nx;
            G[i * w2 + j] = m.Ptil0[e];
            G[i * w2 + nx + j] = i == j ? 1.0 : 0.0;
        }
        wfence();
        const bool ok = gauss_jordan(G, nx);
        for (int e = l; e < nu * nu; e += WT) {
            const int i = e / nu, j = e % nu;
            Qw[e] = (i < nx && j < nx) ? G[i * w2 + nx + j] : (i == j ? 1.0 : 0.0);
        }
        for (int e = l; e < nx * nu; e += WT) {
            const int i = e / nu, j = e % nu;
            if (Qxw) Qxw[e] = 0.0;
            B[e] = i == j ? 1.0 : 0.0;
        }
        for (int e = l; e < nx * nx; e += WT) {
            const int i = e / nx, j = e % nx;
            Qx[e] = 0.0;
            A[e] = i == j ? 1.0 : 0.0;
            const_cast<double *>(o.QxN)[e] = 0.0;
        }
        for (int i = l; i < nx; i += WT) {
            a[i] = 0.0;
            lx[i] = 0.0;
            const_cast<double *>(o.lN)[i] = 0.0;
            const_cast<double *>(o.x0)[i] = m.xtil0[i];
        }
        for (int i = l; i < nu; i += WT) lw[i] = 0.0;
        if (l == 0) {
            c[0] = 0.0;
            const_cast<double *>(o.cN)[0] = 0.0;
            if (!ok && info) {
                if (atomicCAS(&info[0], 0, STATUS_NOT_SPD) == 0) info[1] = -1;
            }
        }
        return;
    }
    const int k = t - 1;                   // MHE sample
    const int w2 = 2 * d;
    // [Sigma | I] with Sigma = [[Q_w, Q_wv], [Q_wv', Q_v]]
    for (int e = l; e < d * d; e += WT) {
        const int i = e / d, j = e % d;
        double v;
        if (i < nw && j < nw)
            v = at(m.Qw, m.sQw, k, i * nw + j);
        else if (i >= nw && j >= nw)
            v = at(m.Qv, m.sQv, k, (i - nw) * ny + (j - nw));
        else if (i < nw)
            v = at(m.Qwv, m.sQwv, k, i * ny + (j - nw));
        else
            v = at(m.Qwv, m.sQwv, k, j * ny + (i - nw));
        G[i * w2 + j] = v;
        G[i * w2 + d + j] = i == j ? 1.0 : 0.0;
    }
    for (int i = l; i < ny; i += WT)
        yt[i] = m.y[(int64_t)k * m.sy + i] - at(m.d, m.sd, k, i) - at(m.vtil, m.svtil, k, i);
    for (int i = l; i < nw; i += WT) wt[i] = at(m.wtil, m.swtil, k, i);
    wfence();
    const bool ok = gauss_jordan(G, d);
    // blocks of the inverse: W (nw x nw), S (nw x ny), V (ny x ny)
    auto W = [&](int i, int j) { return G[i * w2 + d + j]; };
    auto S = [&](int i, int j) { return G[i * w2 + d + nw + j]; };
    auto V = [&](int i, int j) { return G[(nw + i) * w2 + d + nw + j]; };
    const double *C = m.C + (int64_t)k * m.sC;   // ny x nx
    // T = V C, u = S' wtil - V ytil
    for (int e = l; e < ny * nx; e += WT) {
        const int i = e / nx, j = e % nx;
        double s = 0.0;
        for (int q = 0; q < ny; ++q) s += V(i, q) * C[q * nx + j];
        T[e] = s;
    }
    for (int i = l; i < ny; i += WT) {
        double s = 0.0;
        for (int j = 0; j < nw; ++j) s += S(j, i) * wt[j];
        for (int q = 0; q < ny; ++q) s -= V(i, q) * yt[q];
        u[i] = s;
    }
    wfence();
    for (int e = l; e < nx * nx; e += WT) {
        const int i = e / nx, j = e % nx;
        double s = 0.0;
        for (int q = 0; q < ny; ++q) s += C[q * nx + i] * T[q * nx + j];
        Qx[e] = s;                                        // C' V C
        A[e] = m.A[(int64_t)k * m.sA + e];
    }
    for (int e = l; e < nu * nu; e += WT) {
        const int i = e / nu, j = e % nu;
        Qw[e] = (i < nw && j < nw) ? W(i, j) : (i == j ? 1.0 : 0.0);
    }
    for (int e = l; e < nx * nu; e += WT) {
        const int i = e / nu, j = e % nu;
        if (Qxw) {
            double r = 0.0;                               // -C' S' (zero on the padded inputs)
            if (j < nw)
                for (int q = 0; q < ny; ++q) r += C[q * nx + i] * S(j, q);
            Qxw[e] = -r;
        }
        B[e] = j < nw ? m.B[(int64_t)k * m.sB + i * nw + j] : 0.0;
    }
    double part = 0.0;
    for (int i = l; i < nx; i += WT) {
        double sx = 0.0;
        for (int q = 0; q < ny; ++q) sx += C[q * nx + i] * u[q];
        lx[i] = sx;                                       // C'(S' wtil - V ytil)
        a[i] = at(m.a, m.sa, k, i);
    }
    for (int i = l; i < nu; i += WT) {
        double sw = 0.0, ww = 0.0;
        if (i < nw) {
            for (int q = 0; q < ny; ++q) sw += S(i, q) * yt[q];
            for (int j = 0; j < nw; ++j) ww += W(i, j) * wt[j];
            part += wt[i] * (0.5 * ww - sw);              // 1/2 wtil'W wtil - wtil'S ytil
        }
        lw[i] = sw - ww;                                  // S ytil - W wtil (0 on the padded inputs)
    }
    for (int i = l; i < ny; i += WT) {
        double vy = 0.0;
        for (int q = 0; q < ny; ++q) vy += V(i, q) * yt[q];
        part += 0.5 * yt[i] * vy;                         // 1/2 ytil'V ytil
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    if (l == 0) {
        c[0] = part;
        if (!ok && info) {
            if (atomicCAS(&info[0], 0, STATUS_NOT_SPD) == 0) info[1] = k;
        }
    }
}

}  // namespace mhe
}  // namespace rs

extern "C" rs_status rs_mhe_to_uftoc(int32_t count, const rs_mhe *mhe, const rs_problem *out, void *stream,
                                     int32_t *info_dev) {
    if (count < 1 || !mhe || !out) return RS_ERR_ARG;
    for (int i = 0; i < count; ++i) {
        const rs_mhe &m = mhe[i];
        const rs_problem &o = out[i];
        const int nw = m.nw > 0 ? m.nw : m.nx;
        if (m.nx < 1 || m.ny < 1 || m.nw < 0 || m.nx > rs::mhe::MAXD || nw + m.ny > rs::mhe::MAXD || m.Nmhe < 0)
            return RS_ERR_ARG;
        if (!m.A || !m.B || !m.C || !m.y || !m.Qw || !m.Qv || !m.xtil0 || !m.Ptil0) return RS_ERR_ARG;
        if (o.nx != m.nx || o.nu != (m.nx > nw ? m.nx : nw) || o.N != m.Nmhe + 2) return RS_ERR_ARG;
        if (!o.Qx || !o.Qw || !o.A || !o.B || !o.a || !o.lx || !o.lw || !o.c || !o.QxN || !o.lN || !o.cN || !o.x0)
            return RS_ERR_ARG;
        if (m.Qwv && !o.Qxw) return RS_ERR_ARG;        // correlated noise gives a cross term
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    for (int i = 0; i < count; ++i) {
        const rs_mhe &m = mhe[i];
        const int nw = m.nw > 0 ? m.nw : m.nx, d = nw + m.ny, g = d > m.nx ? d : m.nx;
        const size_t lds = sizeof(double) * (2 * (size_t)g * g + (size_t)m.ny * m.nx + 2 * m.ny + nw);
        hipLaunchKernelGGL(rs::mhe::k_mhe_convert, dim3(m.Nmhe + 2), dim3(rs::mhe::WT), lds, st, m, out[i],
                           info_dev ? info_dev + 2 * i : nullptr);
        if (hipGetLastError() != hipSuccess) return RS_ERR_HIP;
    }
    return RS_OK;
}
