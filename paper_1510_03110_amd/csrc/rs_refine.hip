// FP64 KKT residual and iterative refinement of the mixed-precision solve.
//
// KKT system of P(N) (Sec. 2; unknowns lam_0, x_0, w_0, lam_1, ..., lam_N,
// x_N; the Lagrangian carries +lam_0'(xbar_0 - x_0) and
// +lam_{t+1}'(A_t x_t + B_t w_t + a_t - x_{t+1})), right-hand side r:
//   lam_0 row:      -x_0                                             = -xbar_0
//   x_t row:        Qx x_t + Qxw w_t - lam_t + A' lam_{t+1}           = -lx_t
//   w_t row:        Qxw' x_t + Qw w_t + B' lam_{t+1}                  = -lw_t
//   lam_{t+1} row:  A x_t + B w_t - x_{t+1}                           = -a_t
//   x_N row:        QxN x_N - lam_N                                   = -lN
// The residual rho = r - K z is evaluated blockwise in FP64.  Since r depends
// linearly on the problem's (xbar_0, lx, lw, a, lN) with a minus sign, the
// correction K d = rho is the solve of the same problem with
//   xbar_0' = x_0 - xbar_0,  lx' = lx + (Qx x + Qxw w - lam + A' lam+),
//   lw' = lw + (Qxw' x + Qw w + B' lam+),  a' = a + (A x + B w - x+),
//   lN' = lN + QxN x_N - lam_N,  c' = 0,
// i.e. exactly (-rho) arranged as problem data.  The residual kernel writes
// these into the correction problem and, from the same reads, the objective
// of the current iterate.
//   kr_residual  per leaf (4 wavefronts, stages round-robin): correction data,
//                max |r|, max |rho| and the objective part of the leaf
//   kr_update    per leaf: z += d; max |d| and max |z| per block (x, w, lam)
//   kr_check     per instance: reduces the leaf parts in a fixed order;
//                decides convergence (relative residual <= tol and
//                estimated forward error <= tol/10), writes the statistics,
//                the objective and RS_ERR_NOT_CONVERGED
#include <hip/hip_runtime.h>

#include "rs_launch.hpp"
#include "rs_vec.hpp"

namespace rs {
namespace sv {

constexpr int RT = 256;   // 4 wavefronts per leaf

// Orders the LDS traffic of one wavefront (each wavefront of the residual
// kernel works on its own stages and LDS vectors, so no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NX, int NU>
struct RSmem {
    double x[4][NX], w[4][NU], ln[4][NX];
    double cx[4][NX], cw[4][NU], ax[4][NX], qw[4][NX], bw[4][NX];
    double red[4][4];
};

// R x C row-major matrix held by one wavefront, read with contiguous loads:
// LC = C / 2 lanes share a row, lane l holds columns col() and col() + 1 of
// the rows row(ii) = ii * RPI + l / LC.  From the same registers the
// wavefront forms row sums (M x: a sum over the LC lanes of a row) and
// column sums (M'v: a sum over the RPI lanes that hold one column pair), so
// every matrix of a stage is read from memory once.
template <int R, int C>
struct Tile {
    static constexpr int LC = C / 2, RPI = 64 / LC, NI = R / RPI;
    static_assert(C % 2 == 0 && (LC & (LC - 1)) == 0 && LC <= 64 && R % RPI == 0, "tile shape");
    double m0[NI], m1[NI];

    __device__ static int col() { return 2 * (lane() % LC); }
    __device__ static int row(int ii) { return ii * RPI + lane() / LC; }
    __device__ __forceinline__ void load(const double *M) {
        const int c = col();
#pragma unroll
        for (int ii = 0; ii < NI; ++ii) {
            const int r = row(ii);
            m0[ii] = M ? M[r * C + c] : 0.0;
            m1[ii] = M ? M[r * C + c + 1] : 0.0;
        }
    }
    // Lane partial of M'v for the lane's two columns (summed by colsum()).
    __device__ __forceinline__ void tpart(const double *v, double &p0, double &p1) const {
#pragma unroll
        for (int ii = 0; ii < NI; ++ii) {
            const double vr = v[row(ii)];
            p0 += m0[ii] * vr;
            p1 += m1[ii] * vr;
        }
    }
    // Lane partial of u'M v (no reduction: the caller sums it over the wave).
    __device__ __forceinline__ double bilinear(const double *u, const double *v) const {
        const int c = col();
        const double v0 = v[c], v1 = v[c + 1];
        double s = 0.0;
#pragma unroll
        for (int ii = 0; ii < NI; ++ii) s += u[row(ii)] * (m0[ii] * v0 + m1[ii] * v1);
        return s;
    }
    // y = M v into y[0..R) (written by one lane per row); every lane calls it.
    __device__ __forceinline__ void rowsum(const double *v, double *y) const {
        const int c = col();
        const double v0 = v[c], v1 = v[c + 1];
#pragma unroll
        for (int ii = 0; ii < NI; ++ii) {
            const double s = group_sum<LC>(m0[ii] * v0 + m1[ii] * v1);
            if (lane() % LC == 0) y[row(ii)] = s;
        }
    }
    // Column sums of the lane partials into y[0..C) (all lanes call it).
    __device__ __forceinline__ static void colsum(double p0, double p1, double *y) {
#pragma unroll
        for (int o = LC; o < 64; o <<= 1) {
            p0 += __shfl_xor(p0, o, 64);
            p1 += __shfl_xor(p1, o, 64);
        }
        if (lane() < LC) {
            y[col()] = p0;
            y[col() + 1] = p1;
        }
    }
};

template <int NX, int NU>
__global__ void __launch_bounds__(RT) kr_residual(GroupArgs g) {
    __shared__ RSmem<NX, NU> S;
    const LeafItem it = load_leaf(g.leaves, blockIdx.x);
    if (skip_inst(g, it.inst)) return;
    const Prob p = load_prob(g.probs, it.inst);
    const Prob c = load_prob(g.corr ? g.corr : g.probs, it.inst);   // written only with g.corr
    const int wv = (int)(threadIdx.x >> 6), l = lane();
    double rhs = 0.0, res = 0.0, obj = 0.0, zn = 0.0;
    double *xs = S.x[wv], *ws = S.w[wv], *ls = S.ln[wv];
    const int len = uni(it.len);
    using TX = Tile<NX, NX>;      // Q_x, A
    using TU = Tile<NX, NU>;      // Q_xw, B
    using TW = Tile<NU, NU>;      // Q_w (same column pairs per lane as TU)
    for (int s = wv; s < len; s += 4) {
        const int t = it.t0 + s;
        const double *x = p.x + (int64_t)t * NX, *xn = x + NX, *w = p.w + (int64_t)t * NU;
        const double *lam = p.lam + (int64_t)t * NX, *lamn = lam + NX;
        TX mQx, mA;
        TU mQxw, mB;
        TW mQw;
        mQx.load(p.Qx + (int64_t)t * p.sQx);
        mA.load(p.A + (int64_t)t * p.sA);
        mQxw.load(p.Qxw ? p.Qxw + (int64_t)t * p.sQxw : nullptr);
        mB.load(p.B + (int64_t)t * p.sB);
        mQw.load(p.Qw + (int64_t)t * p.sQw);
        const double xi = l < NX ? x[l] : 0.0, wi = l < NU ? w[l] : 0.0;
        const double lami = l < NX ? lam[l] : 0.0, xni = l < NX ? xn[l] : 0.0;
        zn = fmax(zn, fmax(fabs(xi), fmax(fabs(wi), fabs(lami))));
        const double lxi = (l < NX && p.lx) ? p.lx[(int64_t)t * p.slx + l] : 0.0;
        const double lwi = (l < NU && p.lw) ? p.lw[(int64_t)t * p.slw + l] : 0.0;
        const double ai = (l < NX && p.a) ? p.a[(int64_t)t * p.sa + l] : 0.0;
        const double ct = p.c ? p.c[(int64_t)t * p.sc] : 0.0;
        if (l < NX) {
            xs[l] = xi;
            ls[l] = lamn[l];
        }
        if (l < NU) ws[l] = wi;
        wave_sync();
        // Q_x'x + A'lam_{t+1} (x row), Q_xw'x + B'lam_{t+1} + Q_w'w (w row)
        double p0 = 0.0, p1 = 0.0, q0 = 0.0, q1 = 0.0;
        mQx.tpart(xs, p0, p1);
        mA.tpart(ls, p0, p1);
        mQxw.tpart(xs, q0, q1);
        mB.tpart(ls, q0, q1);
        mQw.tpart(ws, q0, q1);
        // objective: 1/2 x'Q_x x + x'Q_xw w + 1/2 w'Q_w w (lane parts)
        double part = 0.5 * mQx.bilinear(xs, xs) + mQxw.bilinear(xs, ws) + 0.5 * mQw.bilinear(ws, ws);
        TX::colsum(p0, p1, S.cx[wv]);
        TU::colsum(q0, q1, S.cw[wv]);
        mA.rowsum(xs, S.ax[wv]);
        mQxw.rowsum(ws, S.qw[wv]);
        mB.rowsum(ws, S.bw[wv]);
        wave_sync();
        if (l < NX) {
            const double dlx = lxi + S.cx[wv][l] + S.qw[wv][l] - lami;
            const double da = ai + S.ax[wv][l] + S.bw[wv][l] - xni;
            if (g.corr) {
                const_cast<double *>(c.lx)[(int64_t)t * c.slx + l] = dlx;
                const_cast<double *>(c.a)[(int64_t)t * c.sa + l] = da;
            }
            rhs = fmax(rhs, fmax(fabs(lxi), fabs(ai)));
            res = fmax(res, fmax(fabs(dlx), fabs(da)));
            part += xi * lxi;
        }
        if (l < NU) {
            const double dlw = lwi + S.cw[wv][l];
            if (g.corr) const_cast<double *>(c.lw)[(int64_t)t * c.slw + l] = dlw;
            rhs = fmax(rhs, fabs(lwi));
            res = fmax(res, fabs(dlw));
            part += wi * lwi;
        }
        obj += wave_sum(part) + ct;
        wave_sync();
    }
    if (wv == 0 && it.t0 == 0) {            // lam_0 row
        if (l < NX) {
            const double d0 = p.x[l] - p.x0[l];
            if (g.corr) const_cast<double *>(c.x0)[l] = d0;
            rhs = fmax(rhs, fabs(p.x0[l]));
            res = fmax(res, fabs(d0));
        }
    }
    if (wv == 1 && (it.flags & LEAF_LAST)) {   // x_N row and the terminal cost
        const int64_t N = it.t0 + len;
        const double *x = p.x + N * NX, *lam = p.lam + N * NX;
        Op<NX, NX> oQ;
        oQ.template load<false>(p.QxN, NX);
        if (l < NX) xs[l] = x[l];
        wave_sync();
        const double qx = oQ.apply(xs);
        double part = 0.0;
        if (l < NX) {
            const double lNi = p.lN ? p.lN[l] : 0.0;
            const double dN = lNi + qx - lam[l];
            if (g.corr) const_cast<double *>(c.lN)[l] = dN;
            zn = fmax(zn, fmax(fabs(x[l]), fabs(lam[l])));
            rhs = fmax(rhs, fabs(lNi));
            res = fmax(res, fabs(dN));
            part = x[l] * (0.5 * qx + lNi);
        }
        obj += wave_sum(part) + (p.cN ? p.cN[0] : 0.0);
    }
    rhs = wave_max(rhs);
    res = wave_max(res);
    zn = wave_max(zn);
    if (l == 0) {
        S.red[wv][0] = rhs;
        S.red[wv][1] = res;
        S.red[wv][2] = obj;
        S.red[wv][3] = zn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double* out = g.part + (int64_t)(g.leaf_base + blockIdx.x) * PART_N;
        double a = 0.0, b = 0.0, o = 0.0, z = 0.0;
        for (int q = 0; q < 4; ++q) {
            a = fmax(a, S.red[q][0]);
            b = fmax(b, S.red[q][1]);
            o += S.red[q][2];
            z = fmax(z, S.red[q][3]);
        }
        out[PART_RHS] = a;
        out[PART_RES] = b;
        out[PART_OBJ] = o;
        out[PART_ZN] = z;
    }
}

// z += d over the leaf's stages (and x_N, lam_N for the last leaf).
template <int NX, int NU>
__global__ void __launch_bounds__(RT) kr_update(GroupArgs g) {
    __shared__ double red[4][6];
    const LeafItem it = load_leaf(g.leaves, blockIdx.x);
    if (skip_inst(g, it.inst)) return;
    const Prob p = load_prob(g.probs, it.inst);
    const Prob c = load_prob(g.corr, it.inst);
    const int tid = threadIdx.x, wv = tid >> 6, l = lane();
    const int nst = uni(it.len) + ((it.flags & LEAF_LAST) ? 1 : 0);   // x, lam entries
    double m[6] = {0, 0, 0, 0, 0, 0};
    {
        const int64_t b0 = (int64_t)it.t0 * NX, n = (int64_t)nst * NX;
        for (int64_t e = tid; e < n; e += RT) {
            const double dx = c.x[b0 + e], dl = c.lam[b0 + e];
            double xv = p.x[b0 + e], lv = p.lam[b0 + e];
            if (!g.measure_only) {
                xv += dx;
                lv += dl;
                p.x[b0 + e] = xv;
                p.lam[b0 + e] = lv;
            }
            m[0] = fmax(m[0], fabs(dx));
            m[2] = fmax(m[2], fabs(dl));
            m[3] = fmax(m[3], fabs(xv));
            m[5] = fmax(m[5], fabs(lv));
        }
    }
    {
        const int64_t b0 = (int64_t)it.t0 * NU, n = (int64_t)it.len * NU;
        for (int64_t e = tid; e < n; e += RT) {
            const double dw = c.w[b0 + e];
            double wv2 = p.w[b0 + e];
            if (!g.measure_only) {
                wv2 += dw;
                p.w[b0 + e] = wv2;
            }
            m[1] = fmax(m[1], fabs(dw));
            m[4] = fmax(m[4], fabs(wv2));
        }
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) m[q] = wave_max(m[q]);
    if (l == 0)
        for (int q = 0; q < 6; ++q) red[wv][q] = m[q];
    __syncthreads();
    if (tid < 6) {
        double v = 0.0;
        for (int q = 0; q < 4; ++q) v = fmax(v, red[q][tid]);
        g.part[(int64_t)(g.leaf_base + blockIdx.x) * PART_N + PART_DX + tid] = v;
    }
}

// mode 0: start (conv = status != OK, statistics cleared);
// mode 1: after a residual pass (relative residual and objective of the
//         current iterate; converged once a correction has been applied,
//         the residual is <= tol and the estimated forward error <= tol/10);
// mode 2: after an update (correction size, forward-error estimate);
// mode 3: final (RS_ERR_NOT_CONVERGED for instances that did not converge);
// mode 4: report of a direct solve after a residual pass (relative residual
//         and backward error of the returned solution; nothing else);
// mode 5: report after a measuring update (estimated relative forward
//         error = the size of the correction relative to the solution).
// Modes 1 and 4 also form the normwise backward error
// ||r - K z|| / (||K|| ||z|| + ||r||) when the leaves carry ||K|| (K-norm
// pass, report plans), else store -1.
__global__ void kr_check(const InstInfo *tab, int count, const double *part, double *stats, int32_t *conv,
                         int32_t *info, const DevProb *probs, int mode, double tol, int32_t *active, int nactive,
                         int with_knorm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (mode == 0 && i < nactive) active[i] = 0;
    if (i >= count) return;
    double *st = stats + (int64_t)i * ST_N;
    if (mode == 0) {
        conv[i] = (info[2 * i] != STATUS_OK || (probs[i].flags & PROB_SKIP)) ? 1 : 0;
        for (int q = 0; q < ST_N; ++q) st[q] = 0.0;
        st[ST_EST] = 1.0;
        st[ST_DZ] = 1.0;      // the first solve is taken as 100% wrong
        st[ST_BWD] = -1.0;
        return;
    }
    if (mode == 3) {
        st[ST_CONV] = conv[i] ? 1.0 : 0.0;
        if (info[2 * i] == STATUS_OK && !conv[i]) {
            info[2 * i] = STATUS_NOT_CONVERGED;
            info[2 * i + 1] = -1;
        }
        return;
    }
    if (conv[i]) return;
    const InstInfo in = tab[i];
    const double *pp = part + (int64_t)in.first_leaf * PART_N;
    if (mode == 5) {
        double d[3] = {0, 0, 0}, z[3] = {0, 0, 0};
        for (int lf = 0; lf < in.nleaves; ++lf)
            for (int b = 0; b < 3; ++b) {
                d[b] = fmax(d[b], pp[lf * PART_N + PART_DX + b]);
                z[b] = fmax(z[b], pp[lf * PART_N + PART_X + b]);
            }
        double dz = 0.0;
        for (int b = 0; b < 3; ++b) dz = fmax(dz, z[b] > 0.0 ? d[b] / z[b] : d[b]);
        st[ST_EST] = dz;
        st[ST_DZ] = dz;
        return;
    }
    if (mode == 2) {
        double d[3] = {0, 0, 0}, z[3] = {0, 0, 0};
        for (int lf = 0; lf < in.nleaves; ++lf)
            for (int b = 0; b < 3; ++b) {
                d[b] = fmax(d[b], pp[lf * PART_N + PART_DX + b]);
                z[b] = fmax(z[b], pp[lf * PART_N + PART_X + b]);
            }
        double dz = 0.0;
        for (int b = 0; b < 3; ++b) dz = fmax(dz, z[b] > 0.0 ? d[b] / z[b] : d[b]);
        // The correction d_k measures the error of the previous iterate; the
        // error left after applying it is about d_k times the contraction
        // factor of the iteration, estimated as d_k / d_{k-1}.
        const double est = dz * fmin(1.0, dz / fmax(st[ST_DZ], 1e-300));
        st[ST_DZ] = dz;
        st[ST_EST] = est;
        st[ST_ITERS] += 1.0;
        return;
    }
    double rhs = 0.0, res = 0.0, obj = 0.0, zn = 0.0, kn = 1.0;
    for (int lf = 0; lf < in.nleaves; ++lf) {
        rhs = fmax(rhs, pp[lf * PART_N + PART_RHS]);
        res = fmax(res, pp[lf * PART_N + PART_RES]);
        obj += pp[lf * PART_N + PART_OBJ];
        zn = fmax(zn, pp[lf * PART_N + PART_ZN]);
        kn = fmax(kn, pp[lf * PART_N + PART_KN]);    // the lam_0 row sums to 1
    }
    const double rres = rhs > 0.0 ? res / rhs : res;
    st[ST_RRES] = rres;
    if (with_knorm) {
        const double den = kn * zn + rhs;
        st[ST_BWD] = den > 0.0 ? res / den : res;
    }
    if (mode == 4) return;
    if (probs[i].obj) probs[i].obj[0] = obj;
    if (st[ST_ITERS] >= 1.0 && rres <= tol && st[ST_EST] <= 0.1 * tol) conv[i] = 1;
    else if (active) atomicAdd(active, 1);      // the next correction pass has work
}

template <int NX, int NU>
hipError_t launch_residual(const GroupArgs &g, int, hipStream_t st) {
    hipLaunchKernelGGL((kr_residual<NX, NU>), dim3(g.nleaves), dim3(RT), 0, st, g);
    return hipGetLastError();
}
template <int NX, int NU>
hipError_t launch_update(const GroupArgs &g, int, hipStream_t st) {
    hipLaunchKernelGGL((kr_update<NX, NU>), dim3(g.nleaves), dim3(RT), 0, st, g);
    return hipGetLastError();
}

}  // namespace sv

// which: 0 residual, 1 update.
Launcher refine_kernel(int nx, int nu, int which) {
#define RS_REF(a, b)                                                                   \
    if (nx == a && nu == b) return which == 0 ? &sv::launch_residual<a, b> : &sv::launch_update<a, b>;
    RS_REF(16, 16)
    RS_REF(32, 16)
    RS_REF(32, 32)
#undef RS_REF
    return nullptr;
}

hipError_t launch_refine_check(const InstInfo *tab, int count, const double *part, double *stats, int32_t *conv,
                               int32_t *info, const DevProb *probs, int mode, double tol, int32_t *active,
                               int nactive, int with_knorm, hipStream_t st) {
    const int n = count > nactive ? count : nactive;
    hipLaunchKernelGGL(sv::kr_check, dim3((n + 63) / 64), dim3(64), 0, st, tab, count, part, stats, conv, info,
                       probs, mode, tol, active, nactive, with_knorm);
    return hipGetLastError();
}

namespace sv {

// Largest absolute row sum, over the rows that belong to one leaf, of the
// KKT matrix of P(N) (the rows listed at the top of this file): for stage t
// the x_t rows |Qx| + |Qxw| + 1 + |A'|, the w_t rows |Qxw'| + |Qw| + |B'|,
// the lam_{t+1} rows |A| + |B| + 1; the last leaf adds the x_N rows
// |QxN| + 1.  One workgroup per leaf, one stage at a time: threads i < nx
// form the x and lam+ row sums of row i, threads 128 + j (j < nu) the w row
// sum of row j, each reading its rows and columns in a fixed order
// (deterministic).  Writes PART_KN of the leaf.
__global__ void __launch_bounds__(RT) kn_norm(GroupArgs g) {
    __shared__ double red[RT / 64];
    const LeafItem it = load_leaf(g.leaves, blockIdx.x);
    if (skip_inst(g, it.inst)) return;
    const Prob p = load_prob(g.probs, it.inst);
    const int n = g.nx, m = g.nu, tid = threadIdx.x;
    const int len = uni(it.len);
    double mx = 0.0;
    for (int s = 0; s < len; ++s) {
        const int64_t t = it.t0 + s;
        const double *Qx = p.Qx + t * p.sQx, *Qw = p.Qw + t * p.sQw;
        const double *Qxw = p.Qxw ? p.Qxw + t * p.sQxw : nullptr;
        const double *A = p.A + t * p.sA, *B = p.B + t * p.sB;
        if (tid < n) {
            const int i = tid;
            double rx = 1.0, rl = 1.0;
            for (int j = 0; j < n; ++j) {
                rx += fabs(Qx[(int64_t)i * n + j]) + fabs(A[(int64_t)j * n + i]);
                rl += fabs(A[(int64_t)i * n + j]);
            }
            for (int j = 0; j < m; ++j) {
                rl += fabs(B[(int64_t)i * m + j]);
                if (Qxw) rx += fabs(Qxw[(int64_t)i * m + j]);
            }
            mx = fmax(mx, fmax(rx, rl));
        } else if (tid >= 128 && tid < 128 + m) {
            const int j = tid - 128;
            double rw = 0.0;
            for (int k = 0; k < n; ++k) {
                rw += fabs(B[(int64_t)k * m + j]);
                if (Qxw) rw += fabs(Qxw[(int64_t)k * m + j]);
            }
            for (int k = 0; k < m; ++k) rw += fabs(Qw[(int64_t)j * m + k]);
            mx = fmax(mx, rw);
        }
    }
    if ((it.flags & LEAF_LAST) && tid < n) {
        double rN = 1.0;
        for (int j = 0; j < n; ++j) rN += fabs(p.QxN[(int64_t)tid * n + j]);
        mx = fmax(mx, rN);
    }
    mx = wave_max(mx);
    if (lane() == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (tid == 0) {
        double v = 0.0;
        for (int q = 0; q < RT / 64; ++q) v = fmax(v, red[q]);
        g.part[(int64_t)(g.leaf_base + blockIdx.x) * PART_N + PART_KN] = v;
    }
}

// Per-instance report (rs_info layout: rel_resid, bwd_err, est_fwd_err as
// doubles, then refine_iters, bad_stage, status, reserved as int32) from the
// statistics and the status words.  Without statistics only the status
// words are reported and the measures are -1.
__global__ void kr_report(int count, const double *stats, const int32_t *info, int refined, char *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double *d = reinterpret_cast<double *>(out + (int64_t)i * 40);
    int32_t *w = reinterpret_cast<int32_t *>(out + (int64_t)i * 40 + 24);
    if (stats) {
        const double *st = stats + (int64_t)i * ST_N;
        d[0] = st[ST_RRES];
        d[1] = st[ST_BWD];
        d[2] = st[ST_EST];
        w[0] = refined ? (int32_t)st[ST_ITERS] : 0;
    } else {
        d[0] = d[1] = d[2] = -1.0;
        w[0] = 0;
    }
    w[1] = info[2 * i + 1];
    w[2] = info[2 * i];
    w[3] = 0;
}

}  // namespace sv

namespace sv {

// Finite-input check of one leaf's stages (RS_PLAN_CHECK_INPUTS): every
// element of Qx, Qw, Qxw, A, B, a, lx, lw and c of the leaf's stages, and of
// x0 (first leaf) and QxN, lN, cN (last leaf).  The smallest offending place
// of the instance, encoded 0 for x0, t + 1 for stage t and N + 1 for the
// terminal data, goes to first[inst] (atomic minimum).
__device__ __forceinline__ bool finite_block(const double *p, int64_t n, int tid) {
    bool ok = true;
    if (p)
        for (int64_t e = tid; e < n; e += RT) ok = ok && __builtin_isfinite(p[e]);
    return ok;
}

__global__ void __launch_bounds__(RT) kc_scan(GroupArgs g, int32_t *first) {
    __shared__ int bad_s;
    const LeafItem it = load_leaf(g.leaves, blockIdx.x);
    if ((uni(g.probs[it.inst].flags) & PROB_SKIP) != 0) return;
    const Prob p = load_prob(g.probs, it.inst);
    const int64_t n = g.nx, m = g.nu;
    const int tid = threadIdx.x, len = uni(it.len);
    if (tid == 0) bad_s = 0x7fffffff;
    __syncthreads();
    for (int s = 0; s < len; ++s) {
        const int64_t t = it.t0 + s;
        bool ok = finite_block(p.Qx + t * p.sQx, n * n, tid) && finite_block(p.Qw + t * p.sQw, m * m, tid) &&
                  finite_block(p.Qxw ? p.Qxw + t * p.sQxw : nullptr, n * m, tid) &&
                  finite_block(p.A + t * p.sA, n * n, tid) && finite_block(p.B + t * p.sB, n * m, tid) &&
                  finite_block(p.a ? p.a + t * p.sa : nullptr, n, tid) &&
                  finite_block(p.lx ? p.lx + t * p.slx : nullptr, n, tid) &&
                  finite_block(p.lw ? p.lw + t * p.slw : nullptr, m, tid) &&
                  finite_block(p.c ? p.c + t * p.sc : nullptr, 1, tid);
        if (!ok) atomicMin(&bad_s, (int)t + 1);
    }
    if (it.t0 == 0 && !finite_block(p.x0, n, tid)) atomicMin(&bad_s, 0);
    if (it.flags & LEAF_LAST) {
        const bool ok = finite_block(p.QxN, n * n, tid) && finite_block(p.lN, n, tid) && finite_block(p.cN, 1, tid);
        if (!ok) atomicMin(&bad_s, it.t0 + len + 1);
    }
    __syncthreads();
    if (tid == 0 && bad_s != 0x7fffffff) atomicMin(&first[it.inst], bad_s);
}

// Instances with a non-finite input: status RS_ERR_ARG and the place
// (-1 for x0, the stage, N for the terminal data).
__global__ void kc_mark(int count, const int32_t *first, int32_t *info) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count || first[i] == 0x7fffffff) return;
    info[2 * i] = 1;     // RS_ERR_ARG
    info[2 * i + 1] = first[i] - 1;
}

}  // namespace sv

hipError_t launch_scan(const GroupArgs &g, int32_t *first, hipStream_t st) {
    if (g.nleaves < 1) return hipSuccess;
    hipLaunchKernelGGL(sv::kc_scan, dim3(g.nleaves), dim3(sv::RT), 0, st, g, first);
    return hipGetLastError();
}

hipError_t launch_scan_mark(int count, const int32_t *first, int32_t *info, hipStream_t st) {
    hipLaunchKernelGGL(sv::kc_mark, dim3((count + 63) / 64), dim3(64), 0, st, count, first, info);
    return hipGetLastError();
}

hipError_t launch_knorm(const GroupArgs &g, hipStream_t st) {
    if (g.nleaves < 1 || g.nx > 128 || g.nu > 128) return hipSuccess;
    hipLaunchKernelGGL(sv::kn_norm, dim3(g.nleaves), dim3(sv::RT), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_report(int count, const double *stats, const int32_t *info, int refined, void *out,
                         hipStream_t st) {
    hipLaunchKernelGGL(sv::kr_report, dim3((count + 63) / 64), dim3(64), 0, st, count, stats, info, refined,
                       static_cast<char *>(out));
    return hipGetLastError();
}

}  // namespace rs
