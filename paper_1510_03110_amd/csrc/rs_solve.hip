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
#include "rs_vec.hpp"

namespace rs {
namespace sv {

// LDS vectors of one work unit.
template <int NX, int NU>
struct VSmem {
    double Psi[NX], pt[NX], av[NX], d[NX], x[NX];
    double gw[NU], z[NU], kk[NU], wv[NU];
    double v[NX];
    double fk[NU], fl[NU], fa[NX], fv[NX], fb[NX];   // forward-sweep products
};

// Where a backward stage's operands live.  Stored factors are of type TR
// (double, or float for mixed-precision leaves); a P_{t+1} that comes from
// the problem or a parent's message is FP64 (Pn64).
template <class TR>
struct VSrc {
    const TR *Pn;          // P_{t+1}, symmetric
    const double *Pn64;    // used when Pn is null; both null = 0 (Alg. 4 preliminary terminal)
    const TR *Vn;          // V_{t+1}; nullptr = identity (Alg. 4 only)
    const TR *Li, *LT;     // L^{-1}, L^{-T}, row-major NU x NU
    const TR *K;           // NU x NX row-major
    const double *A, *B;   // dynamics (B: NX x NU row-major)
    const double *a, *lx, *lw;
    double c;
};

// One backward stage of the vector recursion.  Psi, cbar (and v for RED) are
// the running state; Psi_t and k_{t+1} are returned in LDS (S.Psi, S.kk) and
// handed to emit(Psi_i, k_i) from lanes i < NX / i < NU.
template <int NX, int NU, bool RED, bool WANTK, class TR, class Emit>
__device__ __forceinline__ void vstage(VSmem<NX, NU> &S, const VSrc<TR> &q, double &cbar, Emit emit) {
    const int l = lane();
    Op<NX, NX> oP, oA, oV;
    Op<NU, NX> oB;
    Op<NU, NU> oLT, oLi;
    Op<NX, NU> oK;
    if (q.Pn)
        oP.template load<false>(q.Pn, NX);
    else
        oP.template load<false>(q.Pn64, NX);
    oB.template load<false>(q.B, NU);
    oLT.template load<false>(q.LT, NU);
    oA.template load<false>(q.A, NX);
    oK.template load<false>(q.K, NX);
    if constexpr (RED || WANTK) oLi.template load<false>(q.Li, NU);
    if constexpr (RED) {
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
        RowOp<NX, NU> rB;      // B again, as contiguous rows (read from cache)
        rB.load(q.B, NU);
        rB.apply(S.kk, [&](int r, double bk) { S.d[r] = S.av[r] + bk; });   // a + B k
        wsync();
        const double dd = l < NX ? S.d[l] : 0.0;
        const double inc = q.Vn ? oV.apply(S.d) : dd;
        if (l < NX) S.v[l] += inc;
        wsync();
    }
}

// One forward stage (Alg. 3): w = K x + k, x_{t+1} = A x + a + B w and, for
// leaves, lam_t = P_t x - Psi_t.  Operands as in VSrc (ROW-read here).
template <int NX, int NU, bool LAM, class TR>
__device__ __forceinline__ void fstage(VSmem<NX, NU> &S, const TR *K, const double *kvec, const double *A,
                                       const double *B, const double *a, const TR *P, const double *Psi,
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
template <int NX, int NU, class TP>
__device__ __forceinline__ double cost_to_go(const VSmem<NX, NU> &S, const TP *P, double cbar) {
    const int l = lane();
    Op<NX, NX> oP;
    oP.template load<false>(P, NX);
    const double px = oP.apply(S.x);
    const double part = l < NX ? S.x[l] * (0.5 * px - S.Psi[l]) : 0.0;
    return wave_sum(part) + cbar;
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

template <int NX, int NU, class TR>
__device__ __forceinline__ VSrc<TR> prob_src(const Prob &p, int t) {
    VSrc<TR> q;
    q.Pn = nullptr;
    q.Pn64 = nullptr;
    q.Vn = nullptr;
    q.A = p.A + (int64_t)t * p.sA;
    q.B = p.B + (int64_t)t * p.sB;
    q.a = p.a ? p.a + (int64_t)t * p.sa : nullptr;
    q.lx = p.lx ? p.lx + (int64_t)t * p.slx : nullptr;
    q.lw = p.lw ? p.lw + (int64_t)t * p.slw : nullptr;
    q.c = p.c ? p.c[(int64_t)t * p.sc] : 0.0;
    return q;
}

template <int NX>
__device__ __forceinline__ VSrc<double> slot_src(const double *sl) {
    const SlotLayout L{NX};
    VSrc<double> q;
    q.Pn = nullptr;
    q.Pn64 = nullptr;
    q.Vn = nullptr;
    q.A = sl + L.A();
    q.B = sl + L.Qw();
    q.a = sl + L.a();
    q.lx = sl + L.lx();
    q.lw = nullptr;
    q.c = sl[L.c()];
    return q;
}

// ------------------------------------------------------------------ leaves
// Leaf solve from the stored preliminary solution of the leaf reduction
// (Alg. 4 with terminal P = 0).  With the leaf's terminal costate
// lam_N = P_hat x_hat_{i+1} - Psi_hat (the master solution, Alg. 6), the
// Riccati quantities of the true terminal follow by superposition, since
// Psi and k are affine in the terminal Psi_N = -lam_N:
//   Psi_t = Psi_0,t - V_t lam_N,   k_{t+1} = k_0,t+1 + L_{t+1} lam_N,
// with V_t = prod (A + B K)' and L_{t+1} = -G^{-1} B' V_{t+1}; P and K do not
// depend on the terminal linear term.  Alg. 3 then reads
//   w_t = K x_t + k_0 + L lam_N,  lam_t = P_t x_t - Psi_0,t + V_t lam_N,
//   x_{t+1} = A x_t + B w_t + a_t.
// The last leaf was reduced with the true terminal, so its records are
// final (no V, L terms).  `rec` gives the stage pointers K, k, P, Psi, V, L.
// LAMN (or lamn_sent at run time): the parent sent lam_N itself (the fused
// matrix-core tree, and the superposition down pass of the stored
// factorization) rather than its cost to go P_hat, Psi_hat.
template <int NX, int NU, bool LAMN = false, class Rec>
__device__ __forceinline__ void leaf_forward_sweep(VSmem<NX, NU> &S, double *lamN, const Prob &p,
                                                   const LeafItem &it, const double *msg, Rec rec,
                                                   bool lamn_sent = false) {
    const SlotLayout SL{NX};
    const bool last = (it.flags & LEAF_LAST) != 0;
    const int l = lane();
    if ((LAMN || lamn_sent) && !last) {
        if (l < NX) lamN[l] = msg[SL.lamN() + l];
        wsync();
    } else if (!last) {
        const double *nxt = msg + SL.size();           // the next leaf's slot: x_hat_{i+1}
        if (l < NX) S.x[l] = nxt[SL.xh() + l];
        wsync();
        Op<NX, NX> oP;
        oP.template load<false>(msg + SL.P(), NX);
        const double lam = oP.apply(S.x) - (l < NX ? msg[SL.Psi() + l] : 0.0);
        if (l < NX) lamN[l] = lam;
        wsync();
    }
    if (l < NX) S.x[l] = msg[SL.xh() + l];
    wsync();
    const int len = uni(it.len);
    for (int s = 0; s < len; ++s) {
        const int t = it.t0 + s;
        // row operands with contiguous loads; P (symmetric) read by columns
        RowOp<NU, NX> rK, rL;
        RowOp<NX, NX> rA, rV;
        RowOp<NX, NU> rB;
        Op<NX, NX> oP;
        rK.load(rec.K(s), NX);
        rA.load(p.A + (int64_t)t * p.sA, NX);
        rB.load(p.B + (int64_t)t * p.sB, NU);
        oP.template load<false>(rec.P(s), NX);
        if (!last) {
            rL.load(rec.L(s), NX);
            rV.load(rec.V(s), NX);
        }
        const double kk = l < NU ? (double)rec.k(s)[l] : 0.0;
        const double psi = l < NX ? (double)rec.Psi(s)[l] : 0.0;
        const double av = (l < NX && p.a) ? p.a[(int64_t)t * p.sa + l] : 0.0;
        rK.apply(S.x, [&](int i, double v) { S.fk[i] = v; });
        rA.apply(S.x, [&](int i, double v) { S.fa[i] = v; });
        if (!last) {
            rL.apply(lamN, [&](int i, double v) { S.fl[i] = v; });
            rV.apply(lamN, [&](int i, double v) { S.fv[i] = v; });
        }
        double lam = oP.apply(S.x) - psi;
        wsync();
        double wv = 0.0;
        if (l < NU) wv = S.fk[l] + kk + (last ? 0.0 : S.fl[l]);
        if (!last && l < NX) lam += S.fv[l];
        if (l < NX) {
            p.x[(int64_t)t * NX + l] = S.x[l];
            p.lam[(int64_t)t * NX + l] = lam;
        }
        if (l < NU) {
            S.wv[l] = wv;
            p.w[(int64_t)t * NU + l] = wv;
        }
        wsync();
        rB.apply(S.wv, [&](int i, double v) { S.fb[i] = v; });
        wsync();
        if (l < NX) S.x[l] = S.fa[l] + av + S.fb[l];
        wsync();
    }
    if (last) {
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

// Stage pointers of a stored-factorization leaf: matrices in the up record
// (type TR), Psi_0 and k_0 in the FP64 vector array.
template <int NX, int NU, class TR>
struct UpRecs {
    const TR *rec;
    const double *vec;
    __device__ const TR *r(int s) const { return rec + (int64_t)s * LeafRec{NX, NU}.per_stage(); }
    __device__ const TR *K(int s) const { return r(s) + LeafRec{NX, NU}.K(); }
    __device__ const TR *P(int s) const { return r(s) + LeafRec{NX, NU}.P(); }
    __device__ const TR *V(int s) const { return r(s) + LeafRec{NX, NU}.V(); }
    __device__ const TR *L(int s) const { return r(s) + LeafRec{NX, NU}.Lt(); }
    __device__ const double *Psi(int s) const { return vec + (int64_t)s * (NX + NU); }
    __device__ const double *k(int s) const { return vec + (int64_t)s * (NX + NU) + NX; }
};

template <int NX, int NU, class TR>
__global__ void __launch_bounds__(WT) kv_leaf_up(GroupArgs g) {
    __shared__ VSmem<NX, NU> S;
    if (pass_idle(g)) return;
    const LeafItem it = load_leaf(g.leaves, blockIdx.x);
    if ((it.flags & LEAF_TOP) || skip_inst(g, it.inst)) return;
    const Prob p = load_prob(g.probs, it.inst);
    const LeafRec R{NX, NU};
    const SlotLayout SL{NX};
    const TR *rec = reinterpret_cast<const TR *>(g.fstore) + g.rec_stage(it.scratch) * (int64_t)R.per_stage();
    double *out = g.slots + (int64_t)it.slot * SL.size();
    const int l = lane();
    const bool last = (it.flags & LEAF_LAST) != 0;
    if (l < NX) {
        S.Psi[l] = (last && p.lN) ? -p.lN[l] : 0.0;
        S.v[l] = 0.0;
    }
    double cbar = (last && p.cN) ? p.cN[0] : 0.0;
    double *vec0 = g.fvec + g.rec_stage(it.scratch) * (int64_t)R.vec();
    wsync();
    for (int s = uni(it.len) - 1; s >= 0; --s) {
        VSrc<TR> q = prob_src<NX, NU, TR>(p, it.t0 + s);
        const TR *r = rec + (int64_t)s * R.per_stage();
        const TR *rn = r + R.per_stage();
        const bool end = s + 1 == it.len;
        q.Li = r + R.L();
        q.LT = r + R.LT();
        q.K = r + R.K();
        // Psi_t and k_{t+1} of this sweep, for the leaf solve
        double *vec = vec0 + (int64_t)s * R.vec();
        auto keep = [&](double psi, double k) {
            if (l < NX) vec[l] = psi;
            if (l < NU) vec[NX + l] = k;
        };
        if (!last) {
            q.Pn = end ? nullptr : rn + R.P();
            q.Vn = end ? nullptr : rn + R.V();
            vstage<NX, NU, true, false>(S, q, cbar, keep);
        } else {
            q.Pn = end ? nullptr : rn + R.P();
            q.Pn64 = end ? p.QxN : nullptr;
            vstage<NX, NU, false, true>(S, q, cbar, keep);
        }
    }
    if (l < NX) {
        if (!last) out[SL.a() + l] = S.v[l];
        out[SL.lx() + l] = -S.Psi[l];
    }
    if (l == 0) out[SL.c()] = cbar;
}

template <int NX, int NU, class TR>
__global__ void __launch_bounds__(WT) kv_leaf_down(GroupArgs g) {
    __shared__ VSmem<NX, NU> S;
    __shared__ double lamN[NX];
    if (pass_idle(g)) return;
    const LeafItem it = load_leaf(g.leaves, blockIdx.x);
    if (skip_inst(g, it.inst)) return;
    const Prob p = load_prob(g.probs, it.inst);
    if (!(it.flags & LEAF_TOP)) {
        const int64_t stage0 = g.rec_stage(it.scratch);
        const TR *rec = reinterpret_cast<const TR *>(g.fstore) + stage0 * (int64_t)LeafRec{NX, NU}.per_stage();
        const double *msg = g.slots + (int64_t)it.slot * SlotLayout{NX}.size();
        leaf_forward_sweep<NX, NU>(S, lamN, p, it, msg,
                                   UpRecs<NX, NU, TR>{rec, g.fvec + stage0 * (int64_t)LeafRec{NX, NU}.vec()},
                                   g.superpose != 0);
        return;
    }
    const LeafRec R{NX, NU};
    const SlotLayout SL{NX};
    const int64_t stage0 = g.rec_stage(it.scratch);
    const TR *rec = reinterpret_cast<const TR *>(g.fstore) + stage0 * (int64_t)R.per_stage();
    double *vec0 = g.fvec + stage0 * (int64_t)R.vec();
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
        VSrc<TR> q = prob_src<NX, NU, TR>(p, it.t0 + s);
        const TR *dn = rec + (int64_t)s * R.per_stage() + R.up();
        const bool end = s + 1 == len;
        q.Pn = end ? nullptr : dn + R.per_stage() + R.P();
        q.Pn64 = end ? Pend : nullptr;
        q.Li = dn + R.L();
        q.LT = dn + R.LT();
        q.K = dn + R.K();
        double *vec = vec0 + (int64_t)s * R.vec();
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
        const TR *dn = rec + (int64_t)s * R.per_stage() + R.up();
        const double *vec = vec0 + (int64_t)s * R.vec();
        double lam = 0.0, w = 0.0;
        if (l < NX) p.x[(int64_t)t * NX + l] = S.x[l];
        fstage<NX, NU, true>(S, dn + R.K(), vec + NX, p.A + (int64_t)t * p.sA, p.B + (int64_t)t * p.sB,
                             p.a ? p.a + (int64_t)t * p.sa : nullptr, dn + R.P(), vec, lam, w);
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

// ------------------------------------------- leaf solve of the fused path
// Records of the fused leaf reduction (leaf scratch, FP64 per stage):
//   K (NU*NX) | k (NU) | P (NX*NX) | Psi (NX) | V (NX*NX) | L (NU*NX)
template <int NX, int NU>
struct FusedRecs {
    const double *rec;
    static constexpr int K_ = 0, k_ = NU * NX, P_ = NU * NX + NU, Psi_ = P_ + NX * NX, V_ = Psi_ + NX,
                         L_ = V_ + NX * NX, per = L_ + NU * NX;
    __device__ const double *r(int s) const { return rec + (int64_t)s * per; }
    __device__ const double *K(int s) const { return r(s) + K_; }
    __device__ const double *k(int s) const { return r(s) + k_; }
    __device__ const double *P(int s) const { return r(s) + P_; }
    __device__ const double *Psi(int s) const { return r(s) + Psi_; }
    __device__ const double *V(int s) const { return r(s) + V_; }
    __device__ const double *L(int s) const { return r(s) + L_; }
};

// One wavefront per leaf of a multi-leaf instance (whole-problem leaves are
// solved by the fused leaf-down kernel).
template <int NX, int NU>
__global__ void __launch_bounds__(WT) kv_leaf_fwd(GroupArgs g) {
    __shared__ VSmem<NX, NU> S;
    __shared__ double lamN[NX];
    const LeafItem it = load_leaf(g.leaves, blockIdx.x);
    if ((it.flags & LEAF_TOP) || skip_inst(g, it.inst)) return;
    const Prob p = load_prob(g.probs, it.inst);
    const double *msg = g.slots + (int64_t)it.slot * SlotLayout{NX}.size();
    leaf_forward_sweep<NX, NU, true>(S, lamN, p, it, msg,
                                     FusedRecs<NX, NU>{reinterpret_cast<const double *>(g.leaf_scratch) + it.scratch});
}

template <int NX, int NU>
hipError_t launch_fwd(const GroupArgs &g, int, hipStream_t st) {
    hipLaunchKernelGGL((kv_leaf_fwd<NX, NU>), dim3(g.nleaves), dim3(WT), 0, st, g);
    return hipGetLastError();
}

// -------------------------------------------------------------- the tree
template <int NX>
__global__ void __launch_bounds__(WT) kv_tree(GroupArgs g) {
    __shared__ VSmem<NX, NX> S;
    __shared__ double lamN[NX];
    __shared__ int s_item;
    const int l = lane();
    const SlotLayout SL{NX};
    double *slots = uni_ptr(g.slots);
    auto slot = [&](int s) { return slots + (int64_t)s * SL.size(); };
    if (pass_idle(g)) return;
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
        if (skip_inst(g, it.inst)) {
            // converged: nothing to do (its dependents belong to the same instance)
        } else if (it.kind == ITEM_UP || it.kind == ITEM_UP_LAST) {
            const bool red = it.kind == ITEM_UP;
            const double *term = red ? nullptr : slot(it.term_slot);
            if (l < NX) {
                S.Psi[l] = red ? 0.0 : -term[SL.lx() + l];
                S.v[l] = 0.0;
            }
            double cbar = red ? 0.0 : term[SL.c()];
            wsync();
            for (int s = count - 1; s >= 0; --s) {
                double *sl = slot(it.first + s);
                VSrc<double> q = slot_src<NX>(sl);
                const double *sn = slot(it.first + s + 1);
                const bool end = s + 1 == count;
                q.Li = sl + SL.uL();
                q.LT = sl + SL.uLT();
                q.K = sl + SL.uK();
                // Psi_s and k_s of this sweep, for the superposition sweep down
                auto keep = [&](double psi, double k) {
                    if (g.superpose && l < NX) {
                        sl[SL.Psi() + l] = psi;
                        sl[SL.k() + l] = k;
                    }
                };
                if (red) {
                    q.Pn = end ? nullptr : sn + SL.uP();
                    q.Vn = end ? nullptr : sn + SL.uV();
                    vstage<NX, NX, true, false>(S, q, cbar, keep);
                } else {
                    q.Pn = end ? term + SL.Qx() : sn + SL.uP();
                    q.Vn = nullptr;
                    vstage<NX, NX, false, true>(S, q, cbar, keep);
                }
            }
            double *out = slot(it.out_slot);
            if (l < NX) {
                if (red) out[SL.a() + l] = S.v[l];
                out[SL.lx() + l] = -S.Psi[l];
            }
            if (l == 0) out[SL.c()] = cbar;
        } else if (it.kind == ITEM_DOWN && g.superpose) {
            // Down pass below the top (Alg. 6, k >= 1) as a forward sweep on
            // the records of the item's up pass, with the terminal costate
            // lam_N sent by the parent (the superposition of the leaf solve):
            //   w = K x + k_0 + L_t lam_N,  lam = P x - Psi_0 + V lam_N,
            // x+ = A_hat x + B_hat w + a_hat; the last item of a level holds
            // final records (no lam_N terms).  Child s receives x_s and its
            // terminal costate lam_{s+1}.
            const bool last = it.last != 0;
            const double *msg = slot(it.out_slot);
            if (l < NX) {
                S.x[l] = msg[SL.xh() + l];
                lamN[l] = last ? 0.0 : msg[SL.lamN() + l];
            }
            wsync();
            for (int s = 0; s < count; ++s) {
                double *sl = slot(it.first + s);
                RowOp<NX, NX> rK, rA, rB, rL, rV;
                Op<NX, NX> oP;
                rK.load(sl + SL.uK(), NX);
                rA.load(sl + SL.A(), NX);
                rB.load(sl + SL.Qw(), NX);
                oP.template load<false>(sl + SL.uP(), NX);
                if (!last) {
                    rL.load(sl + SL.dL(), NX);
                    rV.load(sl + SL.uV(), NX);
                }
                const double kk = l < NX ? sl[SL.k() + l] : 0.0;
                const double psi = l < NX ? sl[SL.Psi() + l] : 0.0;
                const double av = l < NX ? sl[SL.a() + l] : 0.0;
                rK.apply(S.x, [&](int i, double v) { S.fk[i] = v; });
                rA.apply(S.x, [&](int i, double v) { S.fa[i] = v; });
                if (!last) {
                    rL.apply(lamN, [&](int i, double v) { S.fl[i] = v; });
                    rV.apply(lamN, [&](int i, double v) { S.fv[i] = v; });
                }
                double lam = oP.apply(S.x) - psi;
                wsync();
                if (l < NX) {
                    if (!last) lam += S.fv[l];
                    sl[SL.xh() + l] = S.x[l];                                    // child s starts at x_s
                    if (s > 0) slot(it.first + s - 1)[SL.lamN() + l] = lam;      // child s-1 ends at lam_s
                    S.wv[l] = S.fk[l] + kk + (last ? 0.0 : S.fl[l]);
                }
                wsync();
                rB.apply(S.wv, [&](int i, double v) { S.fb[i] = v; });
                wsync();
                if (l < NX) S.x[l] = S.fa[l] + av + S.fb[l];
                wsync();
            }
            // the last child ends where the item does: at lam_N, or for the
            // last item at the terminal node, lam = P_term x - Psi_term
            double *lend = slot(it.first + count - 1) + SL.lamN();
            if (last) {
                double *term = slot(it.term_slot);
                Op<NX, NX> oQ;
                oQ.template load<false>(term + SL.Qx(), NX);
                const double v = oQ.apply(S.x);
                if (l < NX) {
                    lend[l] = v + term[SL.lx() + l];
                    term[SL.xh() + l] = S.x[l];
                }
            } else if (l < NX) {
                lend[l] = lamN[l];
            }
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
                VSrc<double> q = slot_src<NX>(sl);
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
                fstage<NX, NX, false, double>(S, sl + SL.K(), sl + SL.k(), sl + SL.A(), sl + SL.Qw(), sl + SL.a(),
                                              nullptr, nullptr, lam, w);
            }
            if (it.last && l < NX) slot(it.term_slot)[SL.xh() + l] = S.x[l];
            if (top && g.superpose) {
                // terminal costate of child s, lam_{s+1} = P_{s+1} x_{s+1} -
                // Psi_{s+1}, from the cost to go sent to it and the initial
                // state of the next child (of the terminal node for the last)
                __threadfence_block();
                wsync();
                for (int s = 0; s < count; ++s) {
                    double *sl = slot(it.first + s);
                    const double *xn = (s + 1 < count ? slot(it.first + s + 1) : slot(it.term_slot)) + SL.xh();
                    if (l < NX) S.fv[l] = xn[l];
                    wsync();
                    Op<NX, NX> oP;
                    oP.template load<false>(sl + SL.P(), NX);
                    const double v = oP.apply(S.fv);
                    if (l < NX) sl[SL.lamN() + l] = v - sl[SL.Psi() + l];
                    wsync();
                }
            }
        }
        __threadfence();
        wsync();
        if (l == 0) __hip_atomic_store(&g.flags[idx], g.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        wsync();
    }
}

template <int NX, int NU, class TR>
hipError_t launch_up(const GroupArgs &g, int, hipStream_t st) {
    hipLaunchKernelGGL((kv_leaf_up<NX, NU, TR>), dim3(g.nleaves), dim3(WT), 0, st, g);
    return hipGetLastError();
}
template <int NX>
hipError_t launch_tree(const GroupArgs &g, int grid, hipStream_t st) {
    hipLaunchKernelGGL((kv_tree<NX>), dim3(grid), dim3(WT), 0, st, g);
    return hipGetLastError();
}
template <int NX, int NU, class TR>
hipError_t launch_down(const GroupArgs &g, int, hipStream_t st) {
    hipLaunchKernelGGL((kv_leaf_down<NX, NU, TR>), dim3(g.nleaves), dim3(WT), 0, st, g);
    return hipGetLastError();
}

}  // namespace sv

Launcher leaf_forward(int nx, int nu) {
    if (nx == 16 && nu == 16) return &sv::launch_fwd<16, 16>;
    if (nx == 32 && nu == 16) return &sv::launch_fwd<32, 16>;
    if (nx == 32 && nu == 32) return &sv::launch_fwd<32, 32>;
    return nullptr;
}

// which: 0 leaf up, 1 tree, 2 leaf down; fp32: the leaf records are FP32.
Launcher vector_solve(int nx, int nu, int which, bool fp32) {
#define RS_VEC(a, b)                                                                   \
    if (nx == a && nu == b) {                                                          \
        if (which == 1) return &sv::launch_tree<a>;                                    \
        if (which == 0) return fp32 ? &sv::launch_up<a, b, float> : &sv::launch_up<a, b, double>; \
        return fp32 ? &sv::launch_down<a, b, float> : &sv::launch_down<a, b, double>; \
    }
    RS_VEC(16, 16)
    RS_VEC(32, 16)
    RS_VEC(32, 32)
#undef RS_VEC
    return nullptr;
}

}  // namespace rs
