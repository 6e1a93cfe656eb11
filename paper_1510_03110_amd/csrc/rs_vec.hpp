// Wavefront-level helpers of the matrix-vector kernels (stored-factor
// solve, residual, refinement update): uniform loads, wave reductions and a
// register-held matrix operand for y = M x.
#pragma once
#include <hip/hip_runtime.h>

#include "rs_types.hpp"

namespace rs {
namespace sv {

constexpr int WT = 64;
constexpr int SPIN_LIMIT = 1 << 26;

__device__ __forceinline__ int lane() { return (int)(threadIdx.x & 63); }
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ const double *uni_ptr(const double *q) {
    const uint64_t v = (uint64_t)q;
    const uint32_t lo = (uint32_t)uni((int)(uint32_t)(v & 0xffffffffu)), hi = (uint32_t)uni((int)(uint32_t)(v >> 32));
    return (const double *)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double *uni_ptr(double *q) { return const_cast<double *>(uni_ptr((const double *)q)); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
    return ((int64_t)uni((int)(v >> 32)) << 32) | (uint32_t)uni((int)(v & 0xffffffff));
}

// A double moved between lanes of a row of 16 by a DPP permutation (CTRL is
// the dpp_ctrl code), without the LDS crossbar round trip of ds_bpermute.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false),
                            __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false));
}

// Sum over aligned groups of G consecutive lanes (G a power of two <= 64);
// every lane of a group receives the group's sum.  Inside a row of 16:
// mirror (lane i <- 15 - i) pairs lanes whose indices sum to 15, half mirror
// (i <- 7 - i within each 8) then leaves every quad holding one partial sum
// of each of four disjoint classes that together cover the row, and the two
// quad swaps (xor 1, xor 2) add those up.  Groups wider than a row add the
// rows with lane shuffles.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    static_assert(G >= 1 && G <= 64 && (G & (G - 1)) == 0, "G a power of two <= 64");
    if constexpr (G >= 16) v += dpp_move<0x140>(v);      // row_mirror
    if constexpr (G >= 8) v += dpp_move<0x141>(v);       // row_half_mirror
    if constexpr (G >= 2) v += dpp_move<0xB1>(v);        // quad_perm [1, 0, 3, 2]
    if constexpr (G >= 4) v += dpp_move<0x4E>(v);        // quad_perm [2, 3, 0, 1]
    if constexpr (G >= 32) v += __shfl_xor(v, 16, 64);
    if constexpr (G >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) { return group_sum<64>(v); }

// Matrix operand of one product y = M x with R outputs and C inputs, held in
// registers.  The wavefront is split into 64 / Rp parts (Rp = R rounded up to
// a power of two); part p sums the contiguous input range
// [p*CH, (p+1)*CH) and the parts are combined with lane shuffles.
//   COL: M(i, k) = M[k*ld + i]  (lanes of a part read consecutive words)
//   ROW: M(i, k) = M[i*ld + k]
template <int R, int C>
struct Op {
    static constexpr int Rp = R <= 1 ? 1 : R <= 2 ? 2 : R <= 4 ? 4 : R <= 8 ? 8 : R <= 16 ? 16 : R <= 32 ? 32 : 64;
    static constexpr int SP = 64 / Rp, CH = (C + SP - 1) / SP;
    static_assert(R <= 64, "at most 64 outputs");
    double m[CH];

    template <bool ROW, class U>
    __device__ __forceinline__ void load(const U *M, int ld) {
        const int l = lane(), i = l % Rp, p = l / Rp;
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int k = p * CH + q;
            m[q] = (M && i < R && k < C) ? (double)(ROW ? M[i * ld + k] : M[k * ld + i]) : 0.0;
        }
    }
    // y_i in every lane with lane % Rp == i (meaningful for i < R).
    __device__ __forceinline__ double apply(const double *x) const {
        const int p = lane() / Rp;
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int k = p * CH + q;
            if (k < C) acc += m[q] * x[k];
        }
#pragma unroll
        for (int o = Rp; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
        return acc;
    }
};

// Row-major matrix operand of y = M x read with contiguous loads: LC = C / 2
// lanes share a row, each holding two consecutive columns, so one load
// instruction of the wavefront covers RPI = 64 / LC whole rows (for a dense
// matrix a contiguous block).  apply() sums the LC partial products of a row
// with DPP lane permutations and hands y_i to out(i, y_i) from lane (i mod RPI) LC.
template <int R, int C>
struct RowOp {
    static constexpr int LC = C / 2, RPI = 64 / LC, NI = (R + RPI - 1) / RPI;
    static_assert(C % 2 == 0 && LC >= 1 && LC <= 64 && (LC & (LC - 1)) == 0, "C / 2 a power of two <= 64");
    double m0[NI], m1[NI];

    template <class U>
    __device__ __forceinline__ void load(const U *M, int ld) {
        const int l = lane(), c = 2 * (l % LC), r0 = l / LC;
#pragma unroll
        for (int ii = 0; ii < NI; ++ii) {
            const int row = ii * RPI + r0;
            const bool ok = M && row < R;
            m0[ii] = ok ? (double)M[row * ld + c] : 0.0;
            m1[ii] = ok ? (double)M[row * ld + c + 1] : 0.0;
        }
    }
    template <class Out>
    __device__ __forceinline__ void apply(const double *x, Out out) const {
        const int l = lane(), c = 2 * (l % LC), r0 = l / LC;
        const double x0 = x[c], x1 = x[c + 1];
#pragma unroll
        for (int ii = 0; ii < NI; ++ii) {
            const double p = group_sum<LC>(m0[ii] * x0 + m1[ii] * x1);
            const int row = ii * RPI + r0;
            if (l % LC == 0 && row < R) out(row, p);
        }
    }
};

// LDS-only barrier (global loads and stores stay in flight across it).
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ LeafItem load_leaf(const LeafItem *tab, int i) {
    const LeafItem r = tab[i];
    LeafItem u;
    u.inst = uni(r.inst);
    u.t0 = uni(r.t0);
    u.len = uni(r.len);
    u.flags = uni(r.flags);
    u.slot = uni(r.slot);
    u.m1 = uni(r.m1);
    u.scratch = uni64(r.scratch);
    return u;
}

// Problem descriptor in wave-uniform registers.
struct Prob {
    const double *Qx, *Qw, *Qxw, *A, *B, *QxN, *x0, *a, *lx, *lw, *c, *lN, *cN;
    double *x, *w, *lam, *obj;
    int64_t sQx, sQw, sQxw, sA, sB, sa, slx, slw, sc;
};
__device__ __forceinline__ Prob load_prob(const DevProb *tab, int i) {
    const DevProb &d = tab[i];
    Prob p;
    p.Qx = uni_ptr(d.Qx);
    p.Qw = uni_ptr(d.Qw);
    p.Qxw = uni_ptr(d.Qxw);
    p.A = uni_ptr(d.A);
    p.B = uni_ptr(d.B);
    p.QxN = uni_ptr(d.QxN);
    p.x0 = uni_ptr(d.x0);
    p.a = uni_ptr(d.a);
    p.lx = uni_ptr(d.lx);
    p.lw = uni_ptr(d.lw);
    p.c = uni_ptr(d.c);
    p.lN = uni_ptr(d.lN);
    p.cN = uni_ptr(d.cN);
    p.x = uni_ptr(d.x);
    p.w = uni_ptr(d.w);
    p.lam = uni_ptr(d.lam);
    p.obj = uni_ptr(d.obj);
    p.sQx = uni64(d.sQx);
    p.sQw = uni64(d.sQw);
    p.sQxw = uni64(d.sQxw);
    p.sA = uni64(d.sA);
    p.sB = uni64(d.sB);
    p.sa = uni64(d.sa);
    p.slx = uni64(d.slx);
    p.slw = uni64(d.slw);
    p.sc = uni64(d.sc);
    return p;
}

// Nothing to do in this refinement pass: every instance has converged.
__device__ __forceinline__ bool pass_idle(const GroupArgs &g) { return g.active && uni(*g.active) == 0; }

// An instance excluded from the call, or converged in the mixed-precision
// refinement, is skipped.
__device__ __forceinline__ bool skip_inst(const GroupArgs &g, int inst) {
    return (uni(g.probs[inst].flags) & PROB_SKIP) != 0 || (g.conv && uni(g.conv[inst]) != 0);
}

}  // namespace sv
}  // namespace rs
