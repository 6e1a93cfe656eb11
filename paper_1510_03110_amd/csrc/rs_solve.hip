// Right-hand-side kernels of the factor / solve split (FP64).
//
// rs_factor stores, for every stage of every level, the matrix results of
// the backward Riccati pass (P_t, L^{-1} and L^{-T} with G_{t+1} = L L', K and,
// for Alg. 4, V_t).  With those the vector lines of Alg. 2-4 and the forward
// recursion of Alg. 3 are matrix-vector products only:
//
//   P a   with P = P_{t+1}           pt  = Psi_{t+1} - P a
//   g_w   = B' pt - l_w             z   = L^{-1} g_w         k = L^{-T} z
//   Psi_t = A' pt + K' g_w - l_x     (K' g_w = -H' G^{-1} g_w, Alg. 2)
//   cbar_t = cbar_{t+1} + 1/2 a'Pa - Psi_{t+1}'a + c - 1/2 z'z
//   Alg. 4:  v += V_{t+1}' (a + B k)
//   Alg. 3:  w = K x + k,  x_{t+1} = A x + B w + a,  lam_t = P_t x - Psi_t
//
// Each work unit (a leaf, a master subproblem) is one wavefront: the
// products are a few hundred multiply-adds, so the unit is bound by the
// latency of its loads, and many independent units per CU hide it.  All
// operands of a stage are loaded into registers before the first product
// of the stage.
//   kv_leaf_up    per leaf: vector part of Alg. 4 / last-leaf elimination
//   kv_tree       work queue over the master levels (vector part of Alg. 5,
//                 top solve, Alg. 6 down to level 1)
//   kv_leaf_down  per leaf: vector part of Alg. 1-2 with the parent's
//                 message, then Alg. 3
#include <hip/hip_runtime.h>

#include "rs_launch.hpp"

namespace rs {
namespace sv {

constexpr int WT = 64;
constexpr int SPIN_LIMIT = 1 << 26;

__device__ __forceinline__ int lane() { return (int)threadIdx.x; }
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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

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

    template <bool ROW>
    __device__ __forceinline__ void load(const double *M, int ld) {
        const int l = lane(), i = l % Rp, p = l / Rp;
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int k = p * CH + q;
            m[q] = (M && i < R && k < C) ? (ROW ? M[i * ld + k] : M[k * ld + i]) : 0.0;
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

__device__ __forceinline__ void wsync() { __syncthreads(); }   // one-wavefront workgroups

// LDS vectors of one work unit.
template <int NX, int NU>
struct VSmem {
    double Psi[NX], pt[NX], av[NX], d[NX], x[NX];
    double gw[NU], z[NU], kk[NU], wv[NU];
    double v[NX];
};

// Where a backward stage's operands live.
struct VSrc {
    const double *Pn;      // P_{t+1}, symmetric; nullptr = 0 (Alg. 4 preliminary terminal)
    const double *Vn;      // V_{t+1}; nullptr = identity (Alg. 4 only)
    const double *A, *B;   // dynamics (B: NX x NU row-major)
    const double *Li, *LT; // L^{-1}, L^{-T}, row-major NU x NU
    const double *K;       // NU x NX row-major
    const double *a, *lx, *lw;
    double c;
};

// One backward stage of the vector recursion.  Psi, cbar (and v for RED) are
// the running state; Psi_t and k_{t+1} are returned in LDS (S.Psi, S.kk) and
// handed to emit(Psi_i, k_i) from lanes i < NX / i < NU.
template <int NX, int NU, bool RED, bool WANTK, class Emit>
__device__ __forceinline__ void vstage(VSmem<NX, NU> &S, const VSrc &q, double &cbar, Emit emit) {
    const int l = lane();
    Op<NX, NX> oP, oA, oV;
    Op<NU, NX> oB;
    Op<NU, NU> oLT, oLi;
    Op<NX, NU> oK, oBr;
    oP.template load<false>(q.Pn, NX);
    oB.template load<false>(q.B, NU);
    oLT.template load<false>(q.LT, NU);
    oA.template load<false>(q.A, NX);
    oK.template load<false>(q.K, NX);
    if constexpr (RED || WANTK) oLi.template load<false>(q.Li, NU);
    if constexpr (RED) {
        oBr.template load<true>(q.B, NU);
        if (q.Vn) oV.template load<false>(q.Vn, NX);
    }
    const double av = (l < NX && q.a) ? q.a[l] : 0.0;
    const double lx = (l < NX && q.lx) ? q.lx[l] : 0.0;
    const double lw = (l < NU && q.lw) ? q.lw[l] : 0.0;
    if (l < NX) S.av[l] = av;
    wsync();
    // P a, pt, cbar += 1/2 a'Pa - Psi'a + c
    {
        const double pa = oP.apply(S.av);
        double part = 0.0;
        if (l < NX) {
            S.pt[l] = S.Psi[l] - pa;
            part = av * (0.5 * pa - S.Psi[l]);
        }
        cbar += wave_sum(part) + q.c;
    }
    wsync();
    {
        const double g = oB.apply(S.pt) - lw;
        if (l < NU) S.gw[l] = g;
    }
    wsync();
    {
        const double z = oLT.apply(S.gw);                        // L^{-1} g_w
        const double psi = oA.apply(S.pt) + oK.apply(S.gw) - lx;  // Psi_t
        if (l < NU) S.z[l] = z;
        cbar -= 0.5 * wave_sum(l < NU ? z * z : 0.0);
        if (l < NX) S.Psi[l] = psi;
    }
    wsync();
    if constexpr (RED || WANTK) {
        const double k = oLi.apply(S.z);                         // L^{-T} z
        if (l < NU) S.kk[l] = k;
        emit(l < NX ? S.Psi[l] : 0.0, k);
        wsync();
    } else {
        emit(l < NX ? S.Psi[l] : 0.0, 0.0);
    }
    if constexpr (RED) {
        const double dd = av + oBr.apply(S.kk);                  // a + B k
        if (l < NX) S.d[l] = dd;
        wsync();
        const double inc = q.Vn ? oV.apply(S.d) : dd;
        if (l < NX) S.v[l] += inc;
        wsync();
    }
}

// One forward stage (Alg. 3): w = K x + k, x_{t+1} = A x + a + B w and, for
// leaves, lam_t = P_t x - Psi_t.  Operands as in VSrc (ROW-read here).
template <int NX, int NU, bool LAM>
__device__ __forceinline__ void fstage(VSmem<NX, NU> &S, const double *K, const double *kvec, const double *A,
                                       const double *B, const double *a, const double *P, const double *Psi,
                                       double &lam_out, double &w_out) {
    const int l = lane();
    Op<NU, NX> oK;
    Op<NX, NX> oA, oP;
    Op<NX, NU> oB;
    oK.template load<true>(K, NX);
    oA.template load<true>(A, NX);
    oB.template load<true>(B, NU);
    if constexpr (LAM) oP.template load<false>(P, NX);
    const double kk = l < NU ? kvec[l] : 0.0;
    const double av = (l < NX && a) ? a[l] : 0.0;
    const double psi = (LAM && l < NX) ? Psi[l] : 0.0;
    const double w = oK.apply(S.x) + kk;
    const double ax = oA.apply(S.x) + av;
    if constexpr (LAM) lam_out = oP.apply(S.x) - psi;
    if (l < NU) S.wv[l] = w;
    w_out = w;
    wsync();
    const double xn = ax + oB.apply(S.wv);
    wsync();
    if (l < NX) S.x[l] = xn;
    wsync();
}

// 1/2 x'Px - Psi'x + cbar (value of the cost to go at x).
template <int NX, int NU>
__device__ __forceinline__ double cost_to_go(const VSmem<NX, NU> &S, const double *P, double cbar) {
    const int l = lane();
    Op<NX, NX> oP;
    oP.template load<false>(P, NX);
    const double px = oP.apply(S.x);
    const double part = l < NX ? S.x[l] * (0.5 * px - S.Psi[l]) : 0.0;
    return wave_sum(part) + cbar;
}

__device__ __forceinline__ LeafItem load_leaf(const LeafItem *tab, int i) {
    const LeafItem r = tab[i];
    LeafItem u;
    u.inst = uni(r.inst);
    u.t0 = uni(r.t0);
    u.len = uni(r.len);
    u.flags = uni(r.flags);
    u.slot = uni(r.slot);
    u.pad = 0;
    u.scratch = uni64(r.scratch);
    return u;
}
__device__ __forceinline__ TreeItem load_item(const TreeItem *tab, int i) {
    const TreeItem r = tab[i];
    TreeItem u;
    u.kind = uni(r.kind);
    u.inst = uni(r.inst);
    u.level = uni(r.level);
    u.first = uni(r.first);
    u.count = uni(r.count);
    u.last = uni(r.last);
    u.term_slot = uni(r.term_slot);
    u.out_slot = uni(r.out_slot);
    u.dep_first = uni(r.dep_first);
    u.dep_count = uni(r.dep_count);
    return u;
}

struct Prob {
    const double *A, *B, *QxN, *x0, *a, *lx, *lw, *c, *lN, *cN;
    double *x, *w, *lam, *obj;
    int64_t sA, sB;
};
__device__ __forceinline__ Prob load_prob(const DevProb *tab, int i) {
    const DevProb &d = tab[i];
    Prob p;
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
    p.sA = uni64(d.sA);
    p.sB = uni64(d.sB);
    return p;
}

template <int NX, int NU>
__device__ __forceinline__ VSrc prob_src(const Prob &p, int t) {
    VSrc q;
    q.A = p.A + (int64_t)t * p.sA;
    q.B = p.B + (int64_t)t * p.sB;
    q.a = p.a ? p.a + (int64_t)t * NX : nullptr;
    q.lx = p.lx ? p.lx + (int64_t)t * NX : nullptr;
    q.lw = p.lw ? p.lw + (int64_t)t * NU : nullptr;
    q.c = p.c ? p.c[t] : 0.0;
    return q;
}

template <int NX>
__device__ __forceinline__ VSrc slot_src(const double *sl) {
    const SlotLayout L{NX};
    VSrc q;
    q.A = sl + L.A();
    q.B = sl + L.Qw();
    q.a = sl + L.a();
    q.lx = sl + L.lx();
    q.lw = nullptr;
    q.c = sl[L.c()];
    return q;
}

// ------------------------------------------------------------------ leaves
template <int NX, int NU>
__global__ void __launch_bounds__(WT) kv_leaf_up(GroupArgs g) {
    __shared__ VSmem<NX, NU> S;
    const LeafItem it = load_leaf(g.leaves, blockIdx.x);
    if (it.flags & LEAF_TOP) return;
    const Prob p = load_prob(g.probs, it.inst);
    const LeafRec R{NX, NU};
    const SlotLayout SL{NX};
    const double *rec = g.fstore + (it.scratch / g.sps) * (int64_t)R.per_stage();
    double *out = g.slots + (int64_t)it.slot * SL.size();
    const int l = lane();
    const bool last = (it.flags & LEAF_LAST) != 0;
    if (l < NX) {
        S.Psi[l] = (last && p.lN) ? -p.lN[l] : 0.0;
        S.v[l] = 0.0;
    }
    double cbar = (last && p.cN) ? p.cN[0] : 0.0;
    wsync();
    auto none = [](double, double) {};
    for (int s = uni(it.len) - 1; s >= 0; --s) {
        VSrc q = prob_src<NX, NU>(p, it.t0 + s);
        const double *r = rec + (int64_t)s * R.per_stage();
        const double *rn = r + R.per_stage();
        const bool end = s + 1 == it.len;
        q.Li = r + R.L();
        q.LT = r + R.LT();
        q.K = r + R.K();
        if (!last) {
            q.Pn = end ? nullptr : rn + R.P();
            q.Vn = end ? nullptr : rn + R.V();
            vstage<NX, NU, true, false>(S, q, cbar, none);
        } else {
            q.Pn = end ? p.QxN : rn + R.P();
            q.Vn = nullptr;
            vstage<NX, NU, false, false>(S, q, cbar, none);
        }
    }
    if (l < NX) {
        if (!last) out[SL.a() + l] = S.v[l];
        out[SL.lx() + l] = -S.Psi[l];
    }
    if (l == 0) out[SL.c()] = cbar;
}

template <int NX, int NU>
__global__ void __launch_bounds__(WT) kv_leaf_down(GroupArgs g) {
    __shared__ VSmem<NX, NU> S;
    const LeafItem it = load_leaf(g.leaves, blockIdx.x);
    const Prob p = load_prob(g.probs, it.inst);
    const LeafRec R{NX, NU};
    const SlotLayout SL{NX};
    double *rec = g.fstore + (it.scratch / g.sps) * (int64_t)R.per_stage();
    const int l = lane();
    const bool known_end = (it.flags & (LEAF_LAST | LEAF_TOP)) != 0;
    const double *msg = (it.flags & LEAF_TOP) ? nullptr : g.slots + (int64_t)it.slot * SL.size();
    const double *Pend = known_end ? p.QxN : msg + SL.P();
    if (l < NX) {
        S.Psi[l] = known_end ? (p.lN ? -p.lN[l] : 0.0) : msg[SL.Psi() + l];
        S.x[l] = msg ? msg[SL.xh() + l] : p.x0[l];
    }
    double cbar = known_end ? (p.cN ? p.cN[0] : 0.0) : msg[SL.cb()];
    wsync();
    const int len = uni(it.len);
    for (int s = len - 1; s >= 0; --s) {
        VSrc q = prob_src<NX, NU>(p, it.t0 + s);
        double *r = rec + (int64_t)s * R.per_stage();
        const double *dn = r + R.up();
        q.Pn = s + 1 == len ? Pend : rec + (int64_t)(s + 1) * R.per_stage() + R.up() + R.P();
        q.Vn = nullptr;
        q.Li = dn + R.L();
        q.LT = dn + R.LT();
        q.K = dn + R.K();
        double *vec = r + R.up() + R.down();
        vstage<NX, NU, false, true>(S, q, cbar, [&](double psi, double k) {
            if (l < NX) vec[l] = psi;
            if (l < NU) vec[NX + l] = k;
        });
    }
    if ((it.flags & LEAF_TOP) && p.obj) {
        const double v = cost_to_go<NX, NU>(S, rec + R.up() + R.P(), cbar);
        if (l == 0) p.obj[0] = v;
    }
    wsync();
    for (int s = 0; s < len; ++s) {
        const int t = it.t0 + s;
        const double *r = rec + (int64_t)s * R.per_stage();
        const double *dn = r + R.up(), *vec = dn + R.down();
        double lam = 0.0, w = 0.0;
        if (l < NX) p.x[(int64_t)t * NX + l] = S.x[l];
        fstage<NX, NU, true>(S, dn + R.K(), vec + NX, p.A + (int64_t)t * p.sA, p.B + (int64_t)t * p.sB,
                             p.a ? p.a + (int64_t)t * NX : nullptr, dn + R.P(), vec, lam, w);
        if (l < NX) p.lam[(int64_t)t * NX + l] = lam;
        if (l < NU) p.w[(int64_t)t * NU + l] = w;
    }
    if (known_end) {
        const int t = it.t0 + len;
        Op<NX, NX> oQ;
        oQ.template load<false>(p.QxN, NX);
        const double lam = oQ.apply(S.x) + ((l < NX && p.lN) ? p.lN[l] : 0.0);
        if (l < NX) {
            p.lam[(int64_t)t * NX + l] = lam;       // lam_N = QxN x_N + lN
            p.x[(int64_t)t * NX + l] = S.x[l];
        }
    }
}

// -------------------------------------------------------------- the tree
template <int NX>
__global__ void __launch_bounds__(WT) kv_tree(GroupArgs g) {
    __shared__ VSmem<NX, NX> S;
    __shared__ int s_item;
    const int l = lane();
    const SlotLayout SL{NX};
    double *slots = uni_ptr(g.slots);
    auto slot = [&](int s) { return slots + (int64_t)s * SL.size(); };
    for (;;) {
        if (l == 0) s_item = atomicAdd(g.queue, 1);
        wsync();
        const int idx = uni(s_item);
        wsync();
        if (idx >= g.nitems) break;
        const TreeItem it = load_item(g.items, idx);
        if (l == 0) {
            for (int d = 0; d < it.dep_count; ++d) {
                int spins = 0;
                while (__hip_atomic_load(&g.flags[it.dep_first + d], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) !=
                       g.epoch) {
                    __builtin_amdgcn_s_sleep(4);
                    if (++spins > SPIN_LIMIT) {
                        int32_t *inf = g.info + 2 * it.inst;
                        atomicCAS(inf, 0, 6);
                        atomicCAS(inf + 1, -1, -2);
                        break;
                    }
                }
            }
        }
        wsync();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int count = it.count;
        if (it.kind == ITEM_UP || it.kind == ITEM_UP_LAST) {
            const bool red = it.kind == ITEM_UP;
            const double *term = red ? nullptr : slot(it.term_slot);
            if (l < NX) {
                S.Psi[l] = red ? 0.0 : -term[SL.lx() + l];
                S.v[l] = 0.0;
            }
            double cbar = red ? 0.0 : term[SL.c()];
            wsync();
            auto none = [](double, double) {};
            for (int s = count - 1; s >= 0; --s) {
                const double *sl = slot(it.first + s);
                VSrc q = slot_src<NX>(sl);
                const double *sn = slot(it.first + s + 1);
                const bool end = s + 1 == count;
                q.Li = sl + SL.uL();
                q.LT = sl + SL.uLT();
                q.K = sl + SL.uK();
                if (red) {
                    q.Pn = end ? nullptr : sn + SL.uP();
                    q.Vn = end ? nullptr : sn + SL.uV();
                    vstage<NX, NX, true, false>(S, q, cbar, none);
                } else {
                    q.Pn = end ? term + SL.Qx() : sn + SL.uP();
                    q.Vn = nullptr;
                    vstage<NX, NX, false, false>(S, q, cbar, none);
                }
            }
            double *out = slot(it.out_slot);
            if (l < NX) {
                if (red) out[SL.a() + l] = S.v[l];
                out[SL.lx() + l] = -S.Psi[l];
            }
            if (l == 0) out[SL.c()] = cbar;
        } else {
            const bool top = it.kind == ITEM_TOP;
            const Prob p = load_prob(g.probs, it.inst);
            const double *msg = top ? nullptr : slot(it.out_slot);
            const double *term = it.last ? slot(it.term_slot) : nullptr;
            if (l < NX) {
                S.Psi[l] = term ? -term[SL.lx() + l] : msg[SL.Psi() + l];
                S.x[l] = top ? p.x0[l] : msg[SL.xh() + l];
            }
            double cbar = term ? term[SL.c()] : msg[SL.cb()];
            wsync();
            for (int s = count - 1; s >= 0; --s) {
                double *sl = slot(it.first + s);
                // message to child s: cost to go at the end of master stage s
                if (l < NX) sl[SL.Psi() + l] = S.Psi[l];
                if (l == 0) sl[SL.cb()] = cbar;
                VSrc q = slot_src<NX>(sl);
                q.Pn = sl + SL.P();
                q.Vn = nullptr;
                q.Li = sl + SL.dL();
                q.LT = sl + SL.dLT();
                q.K = sl + SL.K();
                vstage<NX, NX, false, true>(S, q, cbar, [&](double, double k) {
                    if (l < NX) sl[SL.k() + l] = k;
                });
            }
            if (top && p.obj) {
                const double v = cost_to_go<NX, NX>(S, slot(it.term_slot) + SL.P(), cbar);
                if (l == 0) p.obj[0] = v;
            }
            wsync();
            for (int s = 0; s < count; ++s) {
                double *sl = slot(it.first + s);
                if (l < NX) sl[SL.xh() + l] = S.x[l];
                double lam, w;
                fstage<NX, NX, false>(S, sl + SL.K(), sl + SL.k(), sl + SL.A(), sl + SL.Qw(), sl + SL.a(), nullptr,
                                      nullptr, lam, w);
            }
            if (it.last && l < NX) slot(it.term_slot)[SL.xh() + l] = S.x[l];
        }
        __threadfence();
        wsync();
        if (l == 0) __hip_atomic_store(&g.flags[idx], g.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        wsync();
    }
}

template <int NX, int NU>
hipError_t launch_up(const GroupArgs &g, int, hipStream_t st) {
    hipLaunchKernelGGL((kv_leaf_up<NX, NU>), dim3(g.nleaves), dim3(WT), 0, st, g);
    return hipGetLastError();
}
template <int NX>
hipError_t launch_tree(const GroupArgs &g, int grid, hipStream_t st) {
    hipLaunchKernelGGL((kv_tree<NX>), dim3(grid), dim3(WT), 0, st, g);
    return hipGetLastError();
}
template <int NX, int NU>
hipError_t launch_down(const GroupArgs &g, int, hipStream_t st) {
    hipLaunchKernelGGL((kv_leaf_down<NX, NU>), dim3(g.nleaves), dim3(WT), 0, st, g);
    return hipGetLastError();
}

}  // namespace sv

Launcher vector_solve(int nx, int nu, int which) {
#define RS_VEC(a, b)                                                                   \
    if (nx == a && nu == b) {                                                          \
        if (which == 0) return &sv::launch_up<a, b>;                                   \
        if (which == 1) return &sv::launch_tree<a>;                                    \
        return &sv::launch_down<a, b>;                                                 \
    }
    RS_VEC(16, 16)
    RS_VEC(32, 16)
    RS_VEC(32, 32)
#undef RS_VEC
    return nullptr;
}

}  // namespace rs
