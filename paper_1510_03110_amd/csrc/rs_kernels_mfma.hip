// Matrix-core kernels of the fused parallel Riccati solve for n_x, n_u that
// are multiples of 16 (FP64).  Same work split as the generic kernels:
//   km_leaf_up    one workgroup per leaf: Alg. 4 (or last-leaf elimination)
//   km_tree       work-queue kernel over the master levels (Alg. 5 up, top
//                 solve, Alg. 6 down to level 1)
//   km_leaf_down  one workgroup per leaf: Alg. 1-3 with the parent's message
#include <hip/hip_runtime.h>

#include "rs_launch.hpp"
#include "rs_mfma.hpp"

namespace rs {
namespace mf {

constexpr int SPIN_LIMIT = 1 << 26;

__device__ __forceinline__ LeafItem load_leaf_u(const LeafItem *tab, int i) {
    const LeafItem r = tab[i];
    LeafItem u;
    u.inst = uni(r.inst);
    u.t0 = uni(r.t0);
    u.len = uni(r.len);
    u.flags = uni(r.flags);
    u.slot = uni(r.slot);
    u.m1 = uni(r.m1);
    u.scratch = ((int64_t)uni((int)(r.scratch >> 32)) << 32) | (uint32_t)uni((int)(r.scratch & 0xffffffff));
    return u;
}
__device__ __forceinline__ TreeItem load_item_u(const TreeItem *tab, int i) {
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

template <int NX, int NU>
struct Sizes {
    static constexpr size_t red = sizeof(MSmem<double, NX, NU, true, false>), elim = sizeof(MSmem<double, NX, NU, false, false>),
                            solve = sizeof(MSmem<double, NX, NU, false, true>);
    static constexpr size_t up = red > elim ? red : elim;
    static constexpr size_t all = up > solve ? up : solve;
};

// Reduce (Alg. 4) and write the M1 message.
template <int NX, int NU, class Get, class Out = NoEmit>
__device__ void reduce_to(MSmem<double, NX, NU, true, false> &S, Get get, int count, double *out, int32_t *info, int inst,
                          int stage_base, int fail_code, bool rr, Out emit = Out{}) {
    const int tid = threadIdx.x;
    for (int e = tid; e < NX * NX; e += NT) {
        S.P[e] = 0.0;
        S.V[e] = (e / NX == e % NX) ? 1.0 : 0.0;
        S.Qh[e] = 0.0;
    }
    for (int i = tid; i < NX; i += NT) {
        S.Psi[i] = 0.0;
        S.v[i] = 0.0;
    }
    if (tid == 0) S.cbar = 0.0;
    __syncthreads();
    mfma_pass(S, get, count, info, inst, stage_base, fail_code, [](int, auto &) {}, emit);
    const SlotLayout SL{NX};
    for (int e = tid; e < NX * NX; e += NT) {
        const int i = e / NX, j = e % NX;
        out[SL.A() + e] = S.V[j * NX + i];     // A_hat = V_0'
        if (!rr) out[SL.Qw() + e] = S.Qh[e];
        out[SL.Qx() + e] = S.P[e];
    }
    for (int i = tid; i < NX; i += NT) {
        out[SL.a() + i] = S.v[i];
        out[SL.lx() + i] = -S.Psi[i];
    }
    if (tid == 0) out[SL.c()] = S.cbar;
    if (rr) rank_reveal_rows<NX>(S.Qh, NX, unit_roundoff<double>(), out + SL.Qw(), nullptr);
}

// Eliminate a subproblem with known terminal (already in S) and write the
// terminal cost it passes up (Sec. 4.2, last subproblem).
template <int NX, int NU, class Get, class Out = NoEmit>
__device__ void eliminate_to(MSmem<double, NX, NU, false, false> &S, Get get, int count, double *out, int32_t *info,
                             int inst, int stage_base, int fail_code, Out emit = Out{}) {
    const int tid = threadIdx.x;
    mfma_pass(S, get, count, info, inst, stage_base, fail_code, [](int, auto &) {}, emit);
    const SlotLayout SL{NX};
    for (int e = tid; e < NX * NX; e += NT) out[SL.Qx() + e] = S.P[e];
    for (int i = tid; i < NX; i += NT) out[SL.lx() + i] = -S.Psi[i];
    if (tid == 0) out[SL.c()] = S.cbar;
}

// Forward recursion (Alg. 3) over `count` stages from x in S.x.  Per stage
// the feedback K, k (and for leaves P_t, Psi_t) come from `fac(s)`, the
// dynamics from get(s).  Two barriers per stage; the next stage's operands
// are prefetched into registers and committed to LDS once free.  K, A and B
// are committed transposed so that the lane-per-row products read
// consecutive LDS words; B is double-buffered because it is read in the
// second half.  LDS use: K' in W[0, NU*NX), the second B buffer in
// W[NU*NX, 2*NU*NX), A' in S.A, P in S.P (symmetric).
template <int NX, int NU, bool LAM>
struct FwdPrefetch {
    static constexpr int NK = (NU * NX + NT - 1) / NT, NA = (NX * NX + NT - 1) / NT, NB = (NX * NU + NT - 1) / NT,
                         NP = LAM ? (NX * NX + NT - 1) / NT : 0;
    double k_[NK], a_[NA], b_[NB], p_[NP > 0 ? NP : 1];
    double kk, av, psi;
};

template <int NX, int NU, bool LAM, class Get, class Fac>
__device__ __forceinline__ void fwd_fetch(FwdPrefetch<NX, NU, LAM> &f, Get get, Fac fac, int s) {
    using FP = FwdPrefetch<NX, NU, LAM>;
    const int tid = threadIdx.x;
    const StageSrc src = get(s);
    const double *K = fac.K(s), *P = fac.P(s);
#pragma unroll
    for (int q = 0; q < FP::NK; ++q) {
        const int e = tid + q * NT;
        f.k_[q] = e < NU * NX ? gload(K + e) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < FP::NA; ++q) {
        const int e = tid + q * NT;
        f.a_[q] = e < NX * NX ? gload(src.A + e) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < FP::NB; ++q) {
        const int e = tid + q * NT;
        f.b_[q] = e < NX * NU ? gload(src.B + e) : 0.0;
    }
    if constexpr (LAM) {
#pragma unroll
        for (int q = 0; q < FP::NP; ++q) {
            const int e = tid + q * NT;
            f.p_[q] = e < NX * NX ? gload(P + e) : 0.0;
        }
    }
    f.kk = tid < NU ? gload(fac.k(s) + tid) : 0.0;
    f.av = (tid < NX && src.a) ? gload(src.a + tid) : 0.0;
    f.psi = (LAM && tid < NX) ? gload(fac.Psi(s) + tid) : 0.0;
}

template <int NX, int NU, bool LAM>
__device__ __forceinline__ void fwd_commit_main(MSmem<double, NX, NU, false, true> &S, const FwdPrefetch<NX, NU, LAM> &f) {
    using FP = FwdPrefetch<NX, NU, LAM>;
    const int tid = threadIdx.x;
    double *KT = S.W;
#pragma unroll
    for (int q = 0; q < FP::NK; ++q) {
        const int e = tid + q * NT;        // K[r][c], e = r*NX + c
        if (e < NU * NX) KT[(e % NX) * NU + e / NX] = f.k_[q];
    }
#pragma unroll
    for (int q = 0; q < FP::NA; ++q) {
        const int e = tid + q * NT;        // A[i][c], e = i*NX + c
        if (e < NX * NX) S.A[(e % NX) * NX + e / NX] = f.a_[q];
    }
    if constexpr (LAM) {
#pragma unroll
        for (int q = 0; q < FP::NP; ++q) {
            const int e = tid + q * NT;
            if (e < NX * NX) S.P[e] = f.p_[q];
        }
    }
    if (tid < NU) S.kk[tid] = f.kk;
    if (tid < NX) {
        S.av[tid] = f.av;
        S.Psi[tid] = f.psi;
    }
}

template <int NX, int NU, bool LAM>
__device__ __forceinline__ void fwd_commit_B(double *BT, const FwdPrefetch<NX, NU, LAM> &f) {
    using FP = FwdPrefetch<NX, NU, LAM>;
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < FP::NB; ++q) {
        const int e = tid + q * NT;        // B[i][r], e = i*NU + r
        if (e < NX * NU) BT[(e % NU) * NX + e / NU] = f.b_[q];
    }
}

template <int NX, int NU, bool LAM, class Get, class Fac, class Emit>
__device__ void forward_m(MSmem<double, NX, NU, false, true> &S, Get get, int count, Fac fac, Emit emit) {
    static_assert(2 * NX * NU <= NX * (NX + NU), "K' and the second B buffer live in W");
    const int tid = threadIdx.x;
    count = uni(count);
    FwdPrefetch<NX, NU, LAM> f;
    const double *KT = S.W;
    double *Bcur = S.B, *Bnxt = S.W + NU * NX;
    if (count > 0) {
        fwd_fetch<NX, NU, LAM>(f, get, fac, 0);
        fwd_commit_main<NX, NU, LAM>(S, f);
        fwd_commit_B<NX, NU, LAM>(Bcur, f);
    }
    lds_sync();
    for (int s = 0; s < count; ++s) {
        if (s + 1 < count) fwd_fetch<NX, NU, LAM>(f, get, fac, s + 1);
        // half 1: w = k + K x, A x + a, (leaf) lam = P x - Psi
        if (tid < NU) {
            double acc = S.kk[tid];
#pragma unroll 8
            for (int c = 0; c < NX; ++c) acc += KT[c * NU + tid] * S.x[c];
            S.wv[tid] = acc;
        } else if (tid >= 64 && tid < 64 + NX) {
            const int i = tid - 64;
            double acc = S.av[i];
#pragma unroll 8
            for (int c = 0; c < NX; ++c) acc += S.A[c * NX + i] * S.x[c];
            S.ax[i] = acc;
        } else if (LAM && tid >= 128 && tid < 128 + NX) {
            const int i = tid - 128;
            double acc = -S.Psi[i];
#pragma unroll 8
            for (int c = 0; c < NX; ++c) acc += S.P[c * NX + i] * S.x[c];
            emit.lam(s, i, acc);
        }
        emit.x(s, S.x);
        if (s + 1 < count) fwd_commit_B<NX, NU, LAM>(Bnxt, f);
        lds_sync();
        // half 2: x_{t+1} = A x + a + B w
        if (tid < NX) {
            double acc = S.ax[tid];
#pragma unroll
            for (int r = 0; r < NU; ++r) acc += Bcur[r * NX + tid] * S.wv[r];
            S.x[tid] = acc;
        }
        emit.w(s, S.wv);
        if (s + 1 < count) fwd_commit_main<NX, NU, LAM>(S, f);
        double *t = Bcur;
        Bcur = Bnxt;
        Bnxt = t;
        lds_sync();
    }
}

// Per-stage record of a leaf in the fused solve (leaf scratch), doubles:
//   K_{t+1} (NU*NX) | k_{t+1} (NU) | P_t (NX*NX) | Psi_t (NX) | V_t (NX*NX) | L_{t+1} (NU*NX)
// Written by the leaf reduction: the preliminary solution of Alg. 4 (P = 0
// terminal) with V_t and L_{t+1} = -G^{-1} B' V_{t+1}; for the last leaf (true
// terminal) the first four fields only.  The leaf solve of the whole problem
// (single-leaf instances) writes the first four fields itself.
template <int NX, int NU>
struct LeafFac {
    const double *base;
    static constexpr int K_ = 0, k_ = NU * NX, P_ = NU * NX + NU, Psi_ = NU * NX + NU + NX * NX,
                         V_ = Psi_ + NX, L_ = V_ + NX * NX, per = L_ + NU * NX;
    __device__ const double *K(int s) const { return base + (int64_t)s * per + K_; }
    __device__ const double *k(int s) const { return base + (int64_t)s * per + k_; }
    __device__ const double *P(int s) const { return base + (int64_t)s * per + P_; }
    __device__ const double *Psi(int s) const { return base + (int64_t)s * per + Psi_; }
};

// Writer of those records from the lanes that form each quantity.
template <int NX, int NU, bool RED>
struct LeafRecOut : NoEmit {
    static constexpr bool KF = true, PF = true, VF = RED, LTF = RED, PSF = true, KVF = true;
    double *base;
    using Rec = LeafFac<NX, NU>;
    __device__ double *at(int s) const { return base + (int64_t)s * Rec::per; }
    __device__ void K(int s, int i, int j, double v) const { at(s)[Rec::K_ + i * NX + j] = v; }
    __device__ void k(int s, int i, double v) const { at(s)[Rec::k_ + i] = v; }
    __device__ void P(int s, int i, int j, double v) const { at(s)[Rec::P_ + i * NX + j] = v; }
    __device__ void Psi(int s, int i, double v) const { at(s)[Rec::Psi_ + i] = v; }
    __device__ void V(int s, int i, int j, double v) const { at(s)[Rec::V_ + i * NX + j] = v; }
    __device__ void Lt(int s, int i, int j, double v) const { at(s)[Rec::L_ + i * NX + j] = v; }
};

// ------------------------------------------------------------------ leaves
template <int NX, int NU>
__global__ void __launch_bounds__(NT, 2) km_leaf_up(GroupArgs g) {
    __shared__ __attribute__((aligned(16))) char raw[Sizes<NX, NU>::up];
    const LeafItem it = load_leaf_u(g.leaves, blockIdx.x);
    if ((it.flags & LEAF_TOP) || inst_skipped(g.probs, it.inst)) return;
    const DevProb p = load_prob(g.probs, it.inst);
    const SlotLayout SL{NX};
    double *out = g.slots + (int64_t)it.slot * SL.size();
    auto get = [&](int s) { return prob_stage(p, it.t0 + s); };
    double *rec = reinterpret_cast<double *>(g.leaf_scratch) + it.scratch;
    if (!(it.flags & LEAF_LAST)) {
        auto &S = *reinterpret_cast<MSmem<double, NX, NU, true, false> *>(raw);
        reduce_to<NX, NU>(S, get, it.len, out, g.info, it.inst, it.t0, 2, g.ident != nullptr,
                          LeafRecOut<NX, NU, true>{{}, rec});
    } else {
        auto &S = *reinterpret_cast<MSmem<double, NX, NU, false, false> *>(raw);
        const int tid = threadIdx.x;
        for (int e = tid; e < NX * NX; e += NT) S.P[e] = p.QxN[e];
        for (int i = tid; i < NX; i += NT) S.Psi[i] = p.lN ? -p.lN[i] : 0.0;
        if (tid == 0) S.cbar = p.cN ? p.cN[0] : 0.0;
        __syncthreads();
        eliminate_to<NX, NU>(S, get, it.len, out, g.info, it.inst, it.t0, 2, LeafRecOut<NX, NU, false>{{}, rec});
    }
}

template <int NX, int NU>
__global__ void __launch_bounds__(NT, 3) km_leaf_down(GroupArgs g) {
    __shared__ __attribute__((aligned(16))) char raw[sizeof(MSmem<double, NX, NU, false, true>)];
    auto &S = *reinterpret_cast<MSmem<double, NX, NU, false, true> *>(raw);
    using LF = LeafFac<NX, NU>;
    const LeafItem it = load_leaf_u(g.leaves, blockIdx.x);
    // leaves of multi-leaf instances are finished by the forward sweep on
    // the stored records (leaf_forward)
    if (!(it.flags & LEAF_TOP) || inst_skipped(g.probs, it.inst)) return;
    const DevProb p = load_prob(g.probs, it.inst);
    const SlotLayout SL{NX};
    const int tid = threadIdx.x;
    const bool known_end = (it.flags & (LEAF_LAST | LEAF_TOP)) != 0;
    const double *msg = (it.flags & LEAF_TOP) ? nullptr : g.slots + (int64_t)it.slot * SL.size();
    double *scr = reinterpret_cast<double *>(g.leaf_scratch) + it.scratch;
    for (int e = tid; e < NX * NX; e += NT) S.P[e] = known_end ? p.QxN[e] : msg[SL.P() + e];
    for (int i = tid; i < NX; i += NT) {
        S.Psi[i] = known_end ? (p.lN ? -p.lN[i] : 0.0) : msg[SL.Psi() + i];
        S.x[i] = msg ? msg[SL.xh() + i] : p.x0[i];
    }
    if (tid == 0) S.cbar = known_end ? (p.cN ? p.cN[0] : 0.0) : msg[SL.cb()];
    __syncthreads();
    auto get = [&](int s) { return prob_stage(p, it.t0 + s); };
    struct Out : NoEmit {
        double *scr;
        __device__ double *at(int s) const { return scr + (int64_t)s * LF::per; }
        __device__ void K(int s, int i, int j, double v) const { at(s)[LF::K_ + i * NX + j] = v; }
        __device__ void P(int s, int i, int j, double v) const { at(s)[LF::P_ + i * NX + j] = v; }
        __device__ void Psi(int s, int i, double v) const { at(s)[LF::Psi_ + i] = v; }
        __device__ void k(int s, int i, double v) const { at(s)[LF::k_ + i] = v; }
    };
    mfma_pass(S, get, it.len, g.info, it.inst, it.t0, 2, [](int, auto &) {}, Out{{}, scr});
    if ((it.flags & LEAF_TOP) && p.obj) {
        if (threadIdx.x < 64) {
            double part = 0;
            const int i = threadIdx.x;
            if (i < NX) {
                double acc = 0;
                for (int k = 0; k < NX; ++k) acc += S.P[i * NX + k] * S.x[k];
                part = S.x[i] * (0.5 * acc - S.Psi[i]);
            }
            part = wave_sum(part);
            if (i == 0) p.obj[0] = part + S.cbar;
        }
    }
    __syncthreads();     // scratch written by all threads before it is read back
    struct Emit {
        const DevProb &p;
        int t0;
        __device__ void lam(int s, int i, double v) const { p.lam[(int64_t)(t0 + s) * NX + i] = v; }
        __device__ void x(int s, const double *xv) const {
            const int tid = threadIdx.x;
            if (tid >= 192 && tid < 192 + NX) p.x[(int64_t)(t0 + s) * NX + (tid - 192)] = xv[tid - 192];
        }
        __device__ void w(int s, const double *wv) const {
            const int tid = threadIdx.x;
            if (tid >= 192 && tid < 192 + NU) p.w[(int64_t)(t0 + s) * NU + (tid - 192)] = wv[tid - 192];
        }
    } emit{p, it.t0};
    forward_m<NX, NU, true>(S, get, it.len, LF{scr}, emit);
    if (known_end) {
        const int t = it.t0 + it.len;
        for (int i = tid; i < NX; i += NT) {
            double acc = p.lN ? p.lN[i] : 0.0;
            for (int k = 0; k < NX; ++k) acc += p.QxN[i * NX + k] * S.x[k];
            p.lam[(int64_t)t * NX + i] = acc;       // lam_N = QxN x_N + lN
            p.x[(int64_t)t * NX + i] = S.x[i];
        }
    }
}

// -------------------------------------------------------------- the tree
template <int NX>
struct SlotFac {
    double *slots;
    int first;
    __device__ const double *base(int s) const { return slots + (int64_t)(first + s) * SlotLayout{NX}.size(); }
    __device__ const double *K(int s) const { return base(s) + SlotLayout{NX}.K(); }
    __device__ const double *k(int s) const { return base(s) + SlotLayout{NX}.k(); }
    __device__ const double *P(int s) const { return nullptr; }
    __device__ const double *Psi(int s) const { return nullptr; }
};

// Master feedback K, k of each stage goes to the stage's slot.
template <int NX>
struct SlotOut : NoEmit {
    double *slots;
    int first;
    __device__ double *at(int s) const { return slots + (int64_t)(first + s) * SlotLayout{NX}.size(); }
    __device__ void K(int s, int i, int j, double v) const { at(s)[SlotLayout{NX}.K() + i * NX + j] = v; }
    __device__ void k(int s, int i, double v) const { at(s)[SlotLayout{NX}.k() + i] = v; }
};

// Records of the master stages of an up item (Alg. 4 on the master stages
// with the preliminary terminal; for the last item of a level, the
// elimination with its true terminal), kept in the stages' slots for the down
// sweep: K, k_0, P_t, Psi_0,t and (reduction) V_t, L = -G^{-1} B'V, in the
// slot areas the factored plans use for their up records.
template <int NX, bool RED>
struct SlotRecOut : NoEmit {
    static constexpr bool KF = true, PF = true, VF = RED, LTF = RED, PSF = true, KVF = true;
    double *slots;
    int first;
    __device__ double *at(int s) const { return slots + (int64_t)(first + s) * SlotLayout{NX}.size(); }
    __device__ void K(int s, int i, int j, double v) const { at(s)[SlotLayout{NX}.uK() + i * NX + j] = v; }
    __device__ void k(int s, int i, double v) const { at(s)[SlotLayout{NX}.k() + i] = v; }
    __device__ void P(int s, int i, int j, double v) const { at(s)[SlotLayout{NX}.uP() + i * NX + j] = v; }
    __device__ void Psi(int s, int i, double v) const { at(s)[SlotLayout{NX}.Psi() + i] = v; }
    __device__ void V(int s, int i, int j, double v) const { at(s)[SlotLayout{NX}.uV() + i * NX + j] = v; }
    __device__ void Lt(int s, int i, int j, double v) const { at(s)[SlotLayout{NX}.uL() + i * NX + j] = v; }
};

// Down pass of a master subproblem below the top (Alg. 6, k >= 1) as a
// forward sweep on the records of its up pass, the superposition of the leaf
// solve: with the item's terminal costate lam_N (from its parent),
//   w = K x + k_0 + L lam_N,  lam = P x - Psi_0 + V lam_N,
//   x+ = A_hat x + B_hat w + a_hat;
// the last item of a level holds final records (no lam_N terms) and its
// terminal costate is that of the level's terminal node.  Child s receives
// its initial state x_s and its terminal costate lam_{s+1}.
template <int NX>
__device__ __attribute__((noinline)) void tree_sweep_m(MSmem<double, NX, NX, false, true> &S, const TreeItem &it,
                                                    GroupArgs &g) {
    const SlotLayout SL{NX};
    const int tid = threadIdx.x;
    auto slot = [&](int s) { return g.slots + (int64_t)s * SL.size(); };
    const double *msg = slot(it.out_slot);
    const bool last = it.last != 0;
    double *lamN = S.pt, *lam = S.gx, *xn = S.ax;
    double *Km = S.W, *Lm = S.W + NX * NX, *Vm = S.HT;
    for (int i = tid; i < NX; i += NT) {
        S.x[i] = msg[SL.xh() + i];
        lamN[i] = last ? 0.0 : msg[SL.lamN() + i];
    }
    for (int s = 0; s < it.count; ++s) {
        const double *r = slot(it.first + s);
        const StageSrc src = slot_stage(r, NX, g.ident);
        for (int e = tid; e < NX * NX; e += NT) {
            Km[e] = r[SL.uK() + e];
            S.P[e] = r[SL.uP() + e];
            S.A[e] = src.A[e];
            S.B[e] = src.B[e];
            if (!last) {
                Lm[e] = r[SL.uL() + e];
                Vm[e] = r[SL.uV() + e];
            }
        }
        for (int i = tid; i < NX; i += NT) {
            S.kk[i] = r[SL.k() + i];
            S.Psi[i] = r[SL.Psi() + i];
            S.av[i] = src.a[i];
        }
        __syncthreads();
        if (tid < NX) {
            const int i = tid;
            double w = S.kk[i];
            for (int k = 0; k < NX; ++k) w += Km[i * NX + k] * S.x[k];
            if (!last)
                for (int k = 0; k < NX; ++k) w += Lm[i * NX + k] * lamN[k];
            S.wv[i] = w;
        } else if (tid >= 64 && tid < 64 + NX) {
            const int i = tid - 64;
            double l = -S.Psi[i];
            for (int k = 0; k < NX; ++k) l += S.P[i * NX + k] * S.x[k];
            if (!last)
                for (int k = 0; k < NX; ++k) l += Vm[i * NX + k] * lamN[k];
            lam[i] = l;
        }
        __syncthreads();
        if (tid < NX) {
            const int i = tid;
            double v = S.av[i];
            for (int k = 0; k < NX; ++k) v += S.A[i * NX + k] * S.x[k] + S.B[i * NX + k] * S.wv[k];
            xn[i] = v;
            slot(it.first + s)[SL.xh() + i] = S.x[i];                 // child s starts at x_s
            if (s > 0) slot(it.first + s - 1)[SL.lamN() + i] = lam[i];  // child s-1 ends at lam_s
        }
        __syncthreads();
        if (tid < NX) S.x[tid] = xn[tid];
        __syncthreads();
    }
    // the last child ends where the item does
    if (last) {
        const double *term = slot(it.term_slot);
        if (tid < NX) {
            const int i = tid;
            double l = term[SL.lx() + i];                  // lam_end = P_term x_end - Psi_term
            for (int k = 0; k < NX; ++k) l += term[SL.Qx() + i * NX + k] * S.x[k];
            slot(it.first + it.count - 1)[SL.lamN() + i] = l;
            slot(it.term_slot)[SL.xh() + i] = S.x[i];
        }
    } else if (tid < NX) {
        slot(it.first + it.count - 1)[SL.lamN() + tid] = lamN[tid];
    }
}

template <int NX>
__device__ void tree_solve_m(MSmem<double, NX, NX, false, true> &S, const TreeItem &it, const DevProb &p, GroupArgs &g) {
    const SlotLayout SL{NX};
    const int tid = threadIdx.x;
    double *slots = g.slots;
    auto slot = [&](int s) { return slots + (int64_t)s * SL.size(); };
    const bool top = it.kind == ITEM_TOP;
    const double *msg = top ? nullptr : slot(it.out_slot);
    const double *term = it.last ? slot(it.term_slot) : nullptr;
    for (int e = tid; e < NX * NX; e += NT) S.P[e] = term ? term[SL.Qx() + e] : msg[SL.P() + e];
    for (int i = tid; i < NX; i += NT) {
        S.Psi[i] = term ? -term[SL.lx() + i] : msg[SL.Psi() + i];
        S.x[i] = top ? p.x0[i] : msg[SL.xh() + i];
    }
    if (tid == 0) S.cbar = term ? term[SL.c()] : msg[SL.cb()];
    __syncthreads();
    auto get = [&](int s) { return slot_stage(slot(it.first + s), NX, g.ident); };
    mfma_pass(
        S, get, it.count, g.info, it.inst, -1, 3,
        [&](int s, auto &Sm) {          // M2 for child s: cost to go at the end of stage s
            double *d = slot(it.first + s);
            block_copy<NX * NX>(d + SL.P(), Sm.P);
            if (tid < NX) d[SL.Psi() + tid] = Sm.Psi[tid];
            if (tid == 0) d[SL.cb()] = Sm.cbar;
        },
        SlotOut<NX>{{}, slots, it.first});
    if (top && p.obj && tid < 64) {
        double part = 0;
        if (tid < NX) {
            double acc = 0;
            for (int k = 0; k < NX; ++k) acc += S.P[tid * NX + k] * S.x[k];
            part = S.x[tid] * (0.5 * acc - S.Psi[tid]);
        }
        part = wave_sum(part);
        if (tid == 0) p.obj[0] = part + S.cbar;
    }
    __threadfence_block();
    __syncthreads();
    struct Emit {
        double *slots;
        int first;
        __device__ void lam(int, int, double) const {}
        __device__ void x(int s, const double *xv) const {
            const int tid = threadIdx.x;
            if (tid >= 192 && tid < 192 + NX)
                slots[(int64_t)(first + s) * SlotLayout{NX}.size() + SlotLayout{NX}.xh() + (tid - 192)] = xv[tid - 192];
        }
        __device__ void w(int, const double *) const {}
    } emit{slots, it.first};
    forward_m<NX, NX, false>(S, get, it.count, SlotFac<NX>{slots, it.first}, emit);
    if (it.last) {
        double *d = slot(it.term_slot);
        for (int i = tid; i < NX; i += NT) d[SL.xh() + i] = S.x[i];
    }
    // terminal costate of child s: lam_{s+1} = P_{s+1} x_{s+1} - Psi_{s+1}
    // from the cost to go sent to it and the next child's initial state
    __threadfence_block();
    __syncthreads();
    for (int e = tid; e < it.count * NX; e += NT) {
        const int s = e / NX, i = e - (e / NX) * NX;
        double *d = slot(it.first + s);
        const double *xn = (s + 1 < it.count) ? slot(it.first + s + 1) + SL.xh() : slot(it.term_slot) + SL.xh();
        double l = -d[SL.Psi() + i];
        for (int k = 0; k < NX; ++k) l += d[SL.P() + i * NX + k] * xn[k];
        d[SL.lamN() + i] = l;
    }
}

template <int NX>
__global__ void __launch_bounds__(NT) km_tree(GroupArgs g) {
    __shared__ __attribute__((aligned(16))) char raw[Sizes<NX, NX>::all];
    __shared__ int s_item;
    const int tid = threadIdx.x;
    const SlotLayout SL{NX};
    for (;;) {
        if (tid == 0) s_item = atomicAdd(g.queue, 1);
        __syncthreads();
        const int idx = uni(s_item);
        __syncthreads();
        if (idx >= g.nitems) break;
        const TreeItem it = load_item_u(g.items, idx);
        if (tid == 0) {
            for (int d = 0; d < it.dep_count; ++d) {
                int spins = 0;
                while (__hip_atomic_load(&g.flags[it.dep_first + d], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) !=
                       g.epoch) {
                    __builtin_amdgcn_s_sleep(4);
                    if (++spins > SPIN_LIMIT) {
                        record_failure(g.info, it.inst, 6, -2);
                        break;
                    }
                }
            }
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const DevProb p = load_prob(g.probs, it.inst);
        double *slots = g.slots;
        auto slot = [&](int s) { return slots + (int64_t)s * SL.size(); };
        auto get = [&](int s) { return slot_stage(slot(it.first + s), NX, g.ident); };
        if (inst_skipped(g.probs, it.inst)) {
            // excluded instance: only its completion flag is published
        } else if (it.kind == ITEM_UP) {
            auto &S = *reinterpret_cast<MSmem<double, NX, NX, true, false> *>(raw);
            reduce_to<NX, NX>(S, get, it.count, slot(it.out_slot), g.info, it.inst, -1, 3, g.ident != nullptr,
                              SlotRecOut<NX, true>{{}, slots, it.first});
        } else if (it.kind == ITEM_UP_LAST) {
            auto &S = *reinterpret_cast<MSmem<double, NX, NX, false, false> *>(raw);
            const double *term = slot(it.term_slot);
            for (int e = tid; e < NX * NX; e += NT) S.P[e] = term[SL.Qx() + e];
            for (int i = tid; i < NX; i += NT) S.Psi[i] = -term[SL.lx() + i];
            if (tid == 0) S.cbar = term[SL.c()];
            __syncthreads();
            eliminate_to<NX, NX>(S, get, it.count, slot(it.out_slot), g.info, it.inst, -1, 3,
                                 SlotRecOut<NX, false>{{}, slots, it.first});
        } else if (it.kind == ITEM_TOP) {
            auto &S = *reinterpret_cast<MSmem<double, NX, NX, false, true> *>(raw);
            tree_solve_m<NX>(S, it, p, g);
        } else {
            auto &S = *reinterpret_cast<MSmem<double, NX, NX, false, true> *>(raw);
            tree_sweep_m<NX>(S, it, g);
        }
        __threadfence();
        __syncthreads();
        if (tid == 0) __hip_atomic_store(&g.flags[idx], g.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
    }
}

// ================================================ stored factorization
// rs_factor: the matrix lines of every pass (no right-hand side), writing the
// per-stage factors that rs_solve's vector passes read back.  The leaf passes
// run in T (FP64, or FP32 in mixed-precision plans) and store their records in
// T; the master levels always run in FP64.

// Leaf record writer: up records at +0, down records at +up() of each stage.
template <class T, int NX, int NU, bool UP>
struct LeafFacOut : NoEmit {
    static constexpr bool VEC = false, KF = true, PF = true, LF = true, VF = UP, LTF = UP;
    T *base;                                         // stage 0 of this leaf
    __device__ T *at(int s) const {
        const LeafRec R{NX, NU};
        return base + (int64_t)s * R.per_stage() + (UP ? 0 : R.up());
    }
    __device__ void K(int s, int i, int j, double v) const { at(s)[LeafRec{NX, NU}.K() + i * NX + j] = (T)v; }
    __device__ void P(int s, int i, int j, double v) const { at(s)[LeafRec{NX, NU}.P() + i * NX + j] = (T)v; }
    __device__ void V(int s, int i, int j, double v) const { at(s)[LeafRec{NX, NU}.V() + i * NX + j] = (T)v; }
    __device__ void Lt(int s, int i, int j, double v) const { at(s)[LeafRec{NX, NU}.Lt() + i * NX + j] = (T)v; }
    template <class U>
    __device__ void L(int s, const U *Li) const {
        T *d = at(s);
        const LeafRec R{NX, NU};
        for (int e = threadIdx.x; e < NU * NU; e += NT) {
            const T v = (T)Li[e];
            d[R.L() + e] = v;
            d[R.LT() + (e % NU) * NU + e / NU] = v;
        }
    }
};

// Master-slot writer: up factors (Alg. 4 / elimination) or down factors.
// With `lt` (superposition down pass), the up pass of Alg. 4 also keeps
// L_t = -G^{-1} B' V in the dL place.
template <int NX, bool UP>
struct SlotFacOut : NoEmit {
    static constexpr bool VEC = false, KF = true, PF = UP, LF = true, VF = UP, LTF = UP;
    double *slots;
    int first;
    bool lt;
    __device__ void Lt(int s, int i, int j, double v) const {
        if (lt) at(s)[SlotLayout{NX}.dL() + i * NX + j] = v;
    }
    __device__ double *at(int s) const { return slots + (int64_t)(first + s) * SlotLayout{NX}.size(); }
    __device__ void K(int s, int i, int j, double v) const {
        const SlotLayout L{NX};
        at(s)[(UP ? L.uK() : L.K()) + i * NX + j] = v;
    }
    __device__ void P(int s, int i, int j, double v) const {
        if (UP) at(s)[SlotLayout{NX}.uP() + i * NX + j] = v;
    }
    __device__ void V(int s, int i, int j, double v) const {
        if (UP) at(s)[SlotLayout{NX}.uV() + i * NX + j] = v;
    }
    template <class U>
    __device__ void L(int s, const U *Li) const {
        double *d = at(s);
        const SlotLayout SL{NX};
        const int oL = UP ? SL.uL() : SL.dL(), oT = UP ? SL.uLT() : SL.dLT();
        for (int e = threadIdx.x; e < NX * NX; e += NT) {
            const double v = Li[e];
            d[oL + e] = v;
            d[oT + (e % NX) * NX + e / NX] = v;
        }
    }
};

template <class T, int NX, int NU>
struct FSizes {
    static constexpr size_t red = sizeof(MSmem<T, NX, NU, true, false>), elim = sizeof(MSmem<T, NX, NU, false, false>);
    static constexpr size_t up = red > elim ? red : elim;
};

template <class T, int NX, int NU>
__global__ void __launch_bounds__(NT, 2) kf_leaf_up(GroupArgs g) {
    __shared__ __attribute__((aligned(16))) char raw[FSizes<T, NX, NU>::up];
    const LeafItem it = load_leaf_u(g.leaves, blockIdx.x);
    if ((it.flags & LEAF_TOP) || inst_skipped(g.probs, it.inst)) return;
    const DevProb p = load_prob(g.probs, it.inst);
    const SlotLayout SL{NX};
    double *out = g.slots + (int64_t)it.slot * SL.size();
    T *base = reinterpret_cast<T *>(g.fstore) + g.rec_stage(it.scratch) * (int64_t)LeafRec{NX, NU}.per_stage();
    auto get = [&](int s) { return prob_stage(p, it.t0 + s); };
    const int tid = threadIdx.x;
    if (it.flags & LEAF_REUSE) {
        // stored factorization current (receding-horizon plans): only its
        // cached M1 goes to this call's slot
        const double *c = g.m1cache + (int64_t)it.m1 * 3 * NX * NX;
        for (int e = tid; e < 3 * NX * NX; e += NT) out[e] = c[e];
        return;
    }
    double *cache = (g.m1cache && it.m1 >= 0) ? g.m1cache + (int64_t)it.m1 * 3 * NX * NX : nullptr;
    if (!(it.flags & LEAF_LAST)) {
        auto &S = *reinterpret_cast<MSmem<T, NX, NU, true, false> *>(raw);
        for (int e = tid; e < NX * NX; e += NT) {
            S.P[e] = T(0);
            S.V[e] = (e / NX == e % NX) ? T(1) : T(0);
            S.Qh[e] = T(0);
        }
        __syncthreads();
        mfma_pass(S, get, it.len, g.info, it.inst, it.t0, 2, [](int, auto &) {},
                  LeafFacOut<T, NX, NU, true>{{}, base});
        for (int e = tid; e < NX * NX; e += NT) {
            const int i = e / NX, j = e % NX;
            const double a = S.V[j * NX + i], q = S.Qh[e], x = S.P[e];
            out[SL.A() + e] = a;
            if (!g.ident) out[SL.Qw() + e] = q;
            out[SL.Qx() + e] = x;
            if (cache) {
                cache[SL.A() + e] = a;
                if (!g.ident) cache[SL.Qw() + e] = q;
                cache[SL.Qx() + e] = x;
            }
        }
        if (g.ident) rank_reveal_rows<NX>(S.Qh, NX, unit_roundoff<T>(), out + SL.Qw(), cache ? cache + SL.Qw() : nullptr);
    } else {
        auto &S = *reinterpret_cast<MSmem<T, NX, NU, false, false> *>(raw);
        for (int e = tid; e < NX * NX; e += NT) S.P[e] = (T)p.QxN[e];
        __syncthreads();
        mfma_pass(S, get, it.len, g.info, it.inst, it.t0, 2, [](int, auto &) {},
                  LeafFacOut<T, NX, NU, true>{{}, base});
        for (int e = tid; e < NX * NX; e += NT) out[SL.Qx() + e] = S.P[e];
    }
}

template <class T, int NX, int NU>
__global__ void __launch_bounds__(NT, 3) kf_leaf_down(GroupArgs g) {
    __shared__ __attribute__((aligned(16))) char raw[sizeof(MSmem<T, NX, NU, false, true>)];
    auto &S = *reinterpret_cast<MSmem<T, NX, NU, false, true> *>(raw);
    const LeafItem it = load_leaf_u(g.leaves, blockIdx.x);
    // only whole-problem leaves need the factorization with the true terminal;
    // the others are solved from their up records
    if (!(it.flags & LEAF_TOP) || inst_skipped(g.probs, it.inst)) return;
    const DevProb p = load_prob(g.probs, it.inst);
    const SlotLayout SL{NX};
    const bool known_end = (it.flags & (LEAF_LAST | LEAF_TOP)) != 0;
    const double *msg = (it.flags & LEAF_TOP) ? nullptr : g.slots + (int64_t)it.slot * SL.size();
    T *base = reinterpret_cast<T *>(g.fstore) + g.rec_stage(it.scratch) * (int64_t)LeafRec{NX, NU}.per_stage();
    for (int e = threadIdx.x; e < NX * NX; e += NT) S.P[e] = (T)(known_end ? p.QxN[e] : msg[SL.P() + e]);
    __syncthreads();
    auto get = [&](int s) { return prob_stage(p, it.t0 + s); };
    mfma_pass(S, get, it.len, g.info, it.inst, it.t0, 2, [](int, auto &) {}, LeafFacOut<T, NX, NU, false>{{}, base});
}

template <int NX>
__global__ void __launch_bounds__(NT) kf_tree(GroupArgs g) {
    __shared__ __attribute__((aligned(16))) char raw[Sizes<NX, NX>::all];
    __shared__ int s_item;
    const int tid = threadIdx.x;
    const SlotLayout SL{NX};
    for (;;) {
        if (tid == 0) s_item = atomicAdd(g.queue, 1);
        __syncthreads();
        const int idx = uni(s_item);
        __syncthreads();
        if (idx >= g.nitems) break;
        const TreeItem it = load_item_u(g.items, idx);
        if (tid == 0) {
            for (int d = 0; d < it.dep_count; ++d) {
                int spins = 0;
                while (__hip_atomic_load(&g.flags[it.dep_first + d], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) !=
                       g.epoch) {
                    __builtin_amdgcn_s_sleep(4);
                    if (++spins > SPIN_LIMIT) {
                        record_failure(g.info, it.inst, 6, -2);
                        break;
                    }
                }
            }
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        double *slots = g.slots;
        auto slot = [&](int s) { return slots + (int64_t)s * SL.size(); };
        auto get = [&](int s) { return slot_stage(slot(it.first + s), NX, g.ident); };
        if (inst_skipped(g.probs, it.inst)) {
            // excluded instance: only its completion flag is published
        } else if (it.kind == ITEM_UP) {
            auto &S = *reinterpret_cast<MSmem<double, NX, NX, true, false> *>(raw);
            for (int e = tid; e < NX * NX; e += NT) {
                S.P[e] = 0.0;
                S.V[e] = (e / NX == e % NX) ? 1.0 : 0.0;
                S.Qh[e] = 0.0;
            }
            __syncthreads();
            mfma_pass(S, get, it.count, g.info, it.inst, -1, 3, [](int, auto &) {},
                      SlotFacOut<NX, true>{{}, slots, it.first, g.superpose != 0});
            double *out = slot(it.out_slot);
            for (int e = tid; e < NX * NX; e += NT) {
                const int i = e / NX, j = e % NX;
                out[SL.A() + e] = S.V[j * NX + i];
                if (!g.ident) out[SL.Qw() + e] = S.Qh[e];
                out[SL.Qx() + e] = S.P[e];
            }
            if (g.ident) rank_reveal_rows<NX>(S.Qh, NX, unit_roundoff<double>(), out + SL.Qw(), nullptr);
        } else if (it.kind == ITEM_UP_LAST) {
            auto &S = *reinterpret_cast<MSmem<double, NX, NX, false, false> *>(raw);
            const double *term = slot(it.term_slot);
            for (int e = tid; e < NX * NX; e += NT) S.P[e] = term[SL.Qx() + e];
            __syncthreads();
            mfma_pass(S, get, it.count, g.info, it.inst, -1, 3, [](int, auto &) {},
                      SlotFacOut<NX, true>{{}, slots, it.first, false});
            double *out = slot(it.out_slot);
            for (int e = tid; e < NX * NX; e += NT) out[SL.Qx() + e] = S.P[e];
        } else if (it.kind == ITEM_DOWN && g.superpose) {
            // solved by the vector pass from the up records: nothing to factor
        } else {
            auto &S = *reinterpret_cast<MSmem<double, NX, NX, false, true> *>(raw);
            const bool top = it.kind == ITEM_TOP;
            const double *msg = top ? nullptr : slot(it.out_slot);
            const double *term = it.last ? slot(it.term_slot) : nullptr;
            for (int e = tid; e < NX * NX; e += NT) S.P[e] = term ? term[SL.Qx() + e] : msg[SL.P() + e];
            __syncthreads();
            mfma_pass(
                S, get, it.count, g.info, it.inst, -1, 3,
                [&](int s, auto &Sm) {      // M2 for child s: P at the end of stage s
                    block_copy<NX * NX>(slot(it.first + s) + SL.P(), Sm.P);
                },
                SlotFacOut<NX, false>{{}, slots, it.first, false});
            if (top) block_copy<NX * NX>(slot(it.term_slot) + SL.P(), S.P);   // P_0, for the optimal value
        }
        __threadfence();
        __syncthreads();
        if (tid == 0) __hip_atomic_store(&g.flags[idx], g.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
    }
}

template <int NX, int NU>
hipError_t launch_leaf_up_m(const GroupArgs &g, int, hipStream_t st) {
    hipLaunchKernelGGL((km_leaf_up<NX, NU>), dim3(g.nleaves), dim3(NT), 0, st, g);
    return hipGetLastError();
}
template <int NX>
hipError_t launch_tree_m(const GroupArgs &g, int grid, hipStream_t st) {
    hipLaunchKernelGGL((km_tree<NX>), dim3(grid), dim3(NT), 0, st, g);
    return hipGetLastError();
}
template <int NX, int NU>
hipError_t launch_leaf_down_m(const GroupArgs &g, int grid, hipStream_t st) {
    if (g.ntop > 0) {
        hipLaunchKernelGGL((km_leaf_down<NX, NU>), dim3(g.nleaves), dim3(NT), 0, st, g);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return leaf_forward(NX, NU)(g, grid, st);
}

template <class T, int NX, int NU>
hipError_t launch_factor_leaf_up(const GroupArgs &g, int, hipStream_t st) {
    hipLaunchKernelGGL((kf_leaf_up<T, NX, NU>), dim3(g.nleaves), dim3(NT), 0, st, g);
    return hipGetLastError();
}
template <int NX>
hipError_t launch_factor_tree(const GroupArgs &g, int grid, hipStream_t st) {
    hipLaunchKernelGGL((kf_tree<NX>), dim3(grid), dim3(NT), 0, st, g);
    return hipGetLastError();
}
template <class T, int NX, int NU>
hipError_t launch_factor_leaf_down(const GroupArgs &g, int, hipStream_t st) {
    if (g.ntop == 0) return hipSuccess;
    hipLaunchKernelGGL((kf_leaf_down<T, NX, NU>), dim3(g.nleaves), dim3(NT), 0, st, g);
    return hipGetLastError();
}

}  // namespace mf

// which: 0 leaf up, 1 tree, 2 leaf down; fp32: leaf passes in FP32 (the tree
// is FP64 in both).
Launcher mfma_factor(int nx, int nu, int which, bool fp32) {
#define RS_FAC(a, b)                                                                   \
    if (nx == a && nu == b) {                                                          \
        if (which == 1) return &mf::launch_factor_tree<a>;                             \
        if (which == 0)                                                                \
            return fp32 ? &mf::launch_factor_leaf_up<float, a, b>                     \
                        : &mf::launch_factor_leaf_up<double, a, b>;                   \
        return fp32 ? &mf::launch_factor_leaf_down<float, a, b>                       \
                    : &mf::launch_factor_leaf_down<double, a, b>;                     \
    }
    RS_FAC(16, 16)
    RS_FAC(32, 16)
    RS_FAC(32, 32)
#undef RS_FAC
    return nullptr;
}

// FP32 leaf factorization of the state dimension 64 (mixed precision): the
// FP32 working set of a stage fits in LDS while the FP64 one does not, so
// the leaves run on the matrix-core engine and the master levels and vector
// passes of these shapes on the large-block kernels (same record layouts).
Launcher mfma_factor_leaf32(int nx, int nu, int which) {
    if (nx == 64 && nu == 32)
        return which == 0 ? &mf::launch_factor_leaf_up<float, 64, 32> : &mf::launch_factor_leaf_down<float, 64, 32>;
    if (nx == 64 && nu == 16)
        return which == 0 ? &mf::launch_factor_leaf_up<float, 64, 16> : &mf::launch_factor_leaf_down<float, 64, 16>;
    return nullptr;
}

// MFMA launchers for the shapes that have them (nullptr: use the generic kernel).
Launcher mfma_leaf_up(int nx, int nu) {
    if (nx == 16 && nu == 16) return &mf::launch_leaf_up_m<16, 16>;
    if (nx == 32 && nu == 16) return &mf::launch_leaf_up_m<32, 16>;
    if (nx == 32 && nu == 32) return &mf::launch_leaf_up_m<32, 32>;
    return nullptr;
}
Launcher mfma_leaf_down(int nx, int nu) {
    if (nx == 16 && nu == 16) return &mf::launch_leaf_down_m<16, 16>;
    if (nx == 32 && nu == 16) return &mf::launch_leaf_down_m<32, 16>;
    if (nx == 32 && nu == 32) return &mf::launch_leaf_down_m<32, 32>;
    return nullptr;
}
Launcher mfma_tree(int nx) {
    if (nx == 16) return &mf::launch_tree_m<16>;
    if (nx == 32) return &mf::launch_tree_m<32>;
    return nullptr;
}

}  // namespace rs
