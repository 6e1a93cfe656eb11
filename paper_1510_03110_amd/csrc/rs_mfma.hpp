// Matrix-core (MFMA) version of the per-stage Riccati recursion for state and
// input dimensions that are multiples of 16 (gfx950), in FP64 or FP32: the
// element type T of the working set selects v_mfma_f64_16x16x4f64 or
// v_mfma_f32_16x16x4f32.  Inputs are always read as FP64 and rounded to T
// when staged.
//
// Every dense product of a stage is a list of 16x16 output tiles computed
// by the four wavefronts of the workgroup, tile t going to wave t mod 4.  Operands are read from LDS; products are arranged so
// that the A operand is always read as a transposed (column-contiguous) view,
// which keeps the 16 lanes of one row group on consecutive addresses:
//
//   W   = P [A B]         (P symmetric, so P = P')
//   F   = Qx + A' W_A     H' = Qxw' + B' W_A      G = Qw + B' W_B      (Alg. 1)
//   Y   = L^{-1} H'       z = L^{-1} g_w          (G = L L')
//   P   = F - Y'Y         Psi = g_x - Y'z                              (Alg. 1-2)
//   Alg. 4:  X = L^{-1} B'V,  Q_w_hat += X'X,  V = A'V - Y'X,  v += V'a + X'z
//   solve:   K = -L^{-T} Y,  k = L^{-T} z
//
// Symmetric results (F, P, Q_w_hat) are formed on the lower tiles only and
// mirrored, so they are exactly symmetric.  A stage costs five workgroup
// barriers; the next stage's inputs are prefetched into registers at the
// start of a stage and written to LDS once the current ones are dead.
#pragma once
#include "rs_device.hpp"

namespace rs {
namespace mf {

__device__ __forceinline__ int wave() { return uni((int)(threadIdx.x >> 6)); }
__device__ __forceinline__ int lane() { return (int)(threadIdx.x & 63); }

// The 16x16x4 matrix instruction of each element type.  Operand layout
// (checked on gfx950 for both): A element (i,k) in lane i + 16k, B element
// (k,j) in lane j + 16k.  Result element (row(r), lane%16) in acc[r] with
// row(r) = lane/16 + 4r for f64 and 4(lane/16) + r for f32.
template <class T>
struct MT;
template <>
struct MT<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mfma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int r) { return (lane() >> 4) + 4 * r; }
};
template <>
struct MT<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mfma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int r) { return 4 * (lane() >> 4) + r; }
};
template <class T>
using v4_t = typename MT<T>::v4;
typedef v4_t<double> d4;

// acc += opA[16ti.., k] opB[k, 16tj..] over k < K.  opA(i,k) = TA ? A[k*lda+i]
// : A[i*lda+k]; opB(k,j) = TB ? B[j*ldb+k] : B[k*ldb+j].
// All operand reads of a tile are issued before its first MFMA so that the
// LDS latency is paid once per tile, not once per instruction.
template <int K, bool TA, bool TB, class T>
__device__ __forceinline__ v4_t<T> mma(v4_t<T> acc, const T *__restrict__ A, int lda, const T *__restrict__ B,
                                       int ldb, int ti, int tj) {
    constexpr int S = K / 4;
    const int l = lane(), r16 = l & 15, k4 = l >> 4;
    const int i = 16 * ti + r16, j = 16 * tj + r16;
    T a[S], b[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int k = 4 * s + k4;
        a[s] = TA ? A[k * lda + i] : A[i * lda + k];
        b[s] = TB ? B[j * ldb + k] : B[k * ldb + j];
    }
#pragma unroll
    for (int s = 0; s < S; ++s) acc = MT<T>::mfma(a[s], b[s], acc);
    return acc;
}

// dst[e] = src[e] for e < n (compile-time n), all reads before all writes.
template <int n, class D, class Sx>
__device__ __forceinline__ void block_copy(D *__restrict__ dst, const Sx *__restrict__ src) {
    constexpr int R = (n + NT - 1) / NT;
    const int tid = threadIdx.x;
    double v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int e = tid + q * NT;
        v[q] = (e < n) ? (double)src[e] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int e = tid + q * NT;
        if (e < n) dst[e] = (D)v[q];
    }
}

template <class T = double>
__device__ __forceinline__ v4_t<T> zero4() { return v4_t<T>{T(0), T(0), T(0), T(0)}; }

// Row / column of element r of this lane in tile (ti, tj).
template <class T>
__device__ __forceinline__ int trow(int ti, int r) { return 16 * ti + MT<T>::row(r); }
__device__ __forceinline__ int tcol(int tj) { return 16 * tj + (lane() & 15); }

template <class T, class F>
__device__ __forceinline__ void tile_for(int ti, int tj, F f) {
#pragma unroll
    for (int r = 0; r < 4; ++r) f(r, trow<T>(ti, r), tcol(tj));
}

// Store element (i, j) of a lower tile and its mirror (j, i).  In a diagonal
// tile only the i >= j half writes, so each element has a single writer.
template <class T>
__device__ __forceinline__ void put_sym(T *M, int ld, int ti, int tj, int i, int j, T v) {
    if (ti != tj || i >= j) {
        M[i * ld + j] = v;
        M[j * ld + i] = v;
    }
}

// Lower-triangular tile index t (0 .. T(T+1)/2-1) of a T x T tile grid.
__device__ __forceinline__ void lower_tile(int t, int &ti, int &tj) {
    ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    tj = t - ti * (ti + 1) / 2;
}

// Column of lower-triangular tile t (t = ti (ti + 1) / 2 + tj).
constexpr int lt_col(int t) {
    int ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    return t - ti * (ti + 1) / 2;
}

// The tiles of F, H' and G (phase B enumeration) and the wave that owns each.
// Round robin in general.  For n_u = 16 and n_x <= 32 the first three phases
// are merged (FAST): wave 0 forms G and factors it while wave 1 + tj owns
// column block tj of W_A = P A and the F and H' tiles in that column; then F
// stays in its owner's registers until phase E forms P from it.
template <int NX, int NU>
struct Tiles {
    static constexpr int TX = NX / 16;
    static constexpr int TF = (NX / 16) * (NX / 16 + 1) / 2, TH = (NU / 16) * (NX / 16), TG = (NU / 16) * (NU / 16 + 1) / 2;
    static constexpr int TILES = TF + TH + TG;
    static constexpr bool FAST = NU == 16 && (NX == 16 || NX == 32);
    static constexpr int col(int t) { return t < TF ? lt_col(t) : t < TF + TH ? (t - TF) % TX : 0; }
    static constexpr int owner(int t) { return !FAST ? t % 4 : (t >= TF + TH ? 0 : 1 + col(t)); }
    static constexpr int slot(int t) {
        int n = 0;
        for (int u = 0; u < t; ++u) n += owner(u) == owner(t) ? 1 : 0;
        return n;
    }
    static constexpr int fslot(int t) {        // rank among the owner's F tiles
        int n = 0;
        for (int u = 0; u < t; ++u) n += (u < TF && owner(u) == owner(t)) ? 1 : 0;
        return n;
    }
    static constexpr int max_slots() {
        int m = 0;
        for (int t = 0; t < TILES; ++t) m = slot(t) + 1 > m ? slot(t) + 1 : m;
        return m;
    }
    static constexpr int max_fslots() {
        int m = 1;
        for (int t = 0; t < TF; ++t) m = fslot(t) + 1 > m ? fslot(t) + 1 : m;
        return m;
    }
    static constexpr int PER_WAVE = max_slots(), PER_WAVE_F = max_fslots();
};

// ------------------------------------------------------------------- LDS
template <class T, int NX, int NU, bool RED, bool SOLVE>
struct MSmem {
    typedef T elem;
    static constexpr int NW = NX + NU;
    T P[NX * NX];          // P_{t+1}; F_{t+1} (phase B); P_t (phase E)
    T A[NX * NX];          // stage A_t
    T B[NX * NU];          // stage B_t
    T W[NX * NW];          // P [A B]; then A'V (RED, first NX*NX) and Y (last NU*NX)
    T HT[NU * NX];         // H'
    T G[NU * NU];          // G, then L^{-1} (row-major) with G = L L'
    T LiT[NU * NU];        // L^{-T} (row-major), i.e. L^{-1} by columns
    T V[RED ? NX * NX : 1];
    T Qh[RED ? NX * NX : 1];
    T BV[RED ? NU * NX : 1];   // B'V
    T X[RED ? NU * NX : 1];    // L^{-1} B'V
    T AV[RED && Tiles<NX, NU>::FAST ? NX * NX : 1];   // A'V (merged first phase)
    T Psi[NX], av[NX], lx[NX], pt[NX], pt2[NX], gx[NX], x[NX], ax[NX];
    T lw[NU], gw[NU], z[NU], kk[NU], wv[NU];
    T v[RED ? NX : 1], Vta[RED ? NX : 1];
    T c, cbar, red[4];
    int bad;
    // F is formed in phase B after the last read of P_{t+1} (phase A) and is
    // turned into P_t in place in phase E; Y = L^{-1} H' lives in the part of
    // W that A'V does not use.
    __device__ T *F() { return P; }
    __device__ T *Y() { return W + NX * NX; }
    static_assert(NX * NW >= NX * NX + NU * NX, "Y fits behind A'V in W");
};

// Per-stage results handed out of the pass from the lanes that computed them
// (phase E), and compile-time switches of the pass:
//   VEC  form the vector (right-hand side) quantities of Alg. 2 / Alg. 4
//   KF   form K_{t+1} = -G^{-1} H' also in the reduction (for a later solve)
//   PF, LF, VF  emit P_t, L^{-1} and V_t (stored factorization)
//   LTF  (Alg. 4) form and emit L_{t+1} = -G^{-1} B' V_{t+1} (= -L^{-T} X)
//   PSF, KVF  emit Psi_t and k_{t+1} also outside the solve pass
// The default does nothing and keeps the vector work (fused solve).
struct NoEmit {
    static constexpr bool VEC = true, KF = false, PF = false, LF = false, VF = false, LTF = false, PSF = false,
                          KVF = false;
    __device__ void Lt(int, int, int, double) const {}
    __device__ void K(int, int, int, double) const {}
    __device__ void P(int, int, int, double) const {}
    template <class U>
    __device__ void L(int, const U *) const {}
    __device__ void V(int, int, int, double) const {}
    __device__ void Psi(int, int, double) const {}
    __device__ void k(int, int, double) const {}
};

// Per-thread registers holding the next stage's inputs until they can be
// written to LDS (A, B, a, lx, lw, c) and the tiles of Qx, Qxw', Qw that this
// thread's wave adds in the F / H' / G products.  They hold the FP64 values
// as loaded: a conversion to the working precision at load time would make
// the wave wait for the load right there.
template <class T, int NX, int NU>
struct Prefetch : Tiles<NX, NU> {
    static constexpr int NA = (NX * NX + NT - 1) / NT, NB = (NX * NU + NT - 1) / NT;
    double a_[NA], b_[NB];
    double av, lx, lw, c;
    d4 q[Tiles<NX, NU>::PER_WAVE];
    bool no_qxw;
};

// Waits until every global load and store this wave issued has completed
// (vmcnt(0); expcnt and lgkmcnt left at their maxima).  Issued where the
// only loads still in flight are the next stage's prefetch, started a whole
// phase sequence earlier, so the wait costs little; afterwards no register
// that a phase reads is tied to an outstanding load, and the compiler needs
// no conservative full wait inside the phases (where it would also wait for
// the loads issued at the start of the stage).
__device__ __forceinline__ void wait_global() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Tile t of phase B: F lower tiles, then H' tiles, then G lower tiles.
template <int NX, int NU>
__device__ __forceinline__ void phaseB_tile(int t, int &kind, int &ti, int &tj) {
    using PF = Tiles<NX, NU>;
    if (t < PF::TF) {
        kind = 0;
        lower_tile(t, ti, tj);
    } else if (t < PF::TF + PF::TH) {
        kind = 1;
        const int u = t - PF::TF;
        ti = u / (NX / 16);
        tj = u % (NX / 16);
    } else {
        kind = 2;
        lower_tile(t - PF::TF - PF::TH, ti, tj);
    }
}

// The next stage's A, B and vectors (loaded at the start of a stage) ...
template <class T, int NX, int NU>
__device__ __forceinline__ void prefetch_mats(Prefetch<T, NX, NU> &pf, const StageSrc &s) {
    using PF = Prefetch<T, NX, NU>;
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < PF::NA; ++q) {
        const int e = tid + q * NT;
        pf.a_[q] = e < NX * NX ? gload(s.A + e) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < PF::NB; ++q) {
        const int e = tid + q * NT;
        pf.b_[q] = e < NX * NU ? gload(s.B + e) : 0.0;
    }
    pf.av = (tid < NX && s.a) ? gload(s.a + tid) : 0.0;
    pf.lx = (tid < NX && s.lx) ? gload(s.lx + tid) : 0.0;
    pf.lw = (tid < NU && s.lw) ? gload(s.lw + tid) : 0.0;
    // read through the pointer into the register that holds it until the
    // commit: a copy of an earlier load's result would wait for that load
    pf.c = (tid == 0 && s.cp) ? gload(s.cp) : 0.0;
}

// The phase-B tile held in prefetch slot u by wave w (wave-uniform; false if
// the wave has fewer slots).
template <int NX, int NU>
__device__ __forceinline__ bool slot_tile(int w, int u, int &kind, int &ti, int &tj) {
    using PF = Tiles<NX, NU>;
    bool has = false;
    kind = ti = tj = 0;
#pragma unroll
    for (int t = 0; t < PF::TILES; ++t) {
        int k, a, b;
        phaseB_tile<NX, NU>(t, k, a, b);
        const bool hit = PF::owner(t) == w && PF::slot(t) == u;
        kind = hit ? k : kind;
        ti = hit ? a : ti;
        tj = hit ? b : tj;
        has = has || hit;
    }
    return has;
}

// ... and its Qx / Qxw' / Qw tiles (those of this thread's wave).  Each slot
// register is the destination of one load sequence whose addresses depend on
// the wave: with one sequence per tile instead, the compiler cannot see that
// the waves' sequences exclude each other and makes a later one wait for the
// earlier ones' loads into the same registers.  Without Q_xw the slot reads
// Qx (in bounds) and take_q replaces it with zeros.
template <class T, int NX, int NU>
__device__ __forceinline__ void prefetch_q(Prefetch<T, NX, NU> &pf, const StageSrc &s) {
    using PF = Prefetch<T, NX, NU>;
    const int w = wave(), c = lane() & 15;
#pragma unroll
    for (int u = 0; u < PF::PER_WAVE; ++u) {
        int kind, ti, tj;
        if (!slot_tile<NX, NU>(w, u, kind, ti, tj)) continue;
        const double *base = kind == 0 ? s.Qx : kind == 1 ? (s.Qxw ? s.Qxw : s.Qx) : s.Qw;
        const int si = kind == 0 ? NX : kind == 1 ? 1 : NU, sj = kind == 1 ? NU : 1;
        d4 q;
#pragma unroll
        for (int r = 0; r < 4; ++r) q[r] = gload(base + (16 * ti + MT<T>::row(r)) * si + (16 * tj + c) * sj);
        pf.q[u] = q;
    }
    pf.no_qxw = s.Qxw == nullptr;
}

// The prefetched tiles in the working precision.
template <class T, int NX, int NU>
__device__ __forceinline__ void take_q(v4_t<T> *qt, const Prefetch<T, NX, NU> &pf) {
    const int w = wave();
#pragma unroll
    for (int u = 0; u < Tiles<NX, NU>::PER_WAVE; ++u) {
        int kind, ti, tj;
        const bool zero = slot_tile<NX, NU>(w, u, kind, ti, tj) && kind == 1 && pf.no_qxw;
        qt[u] = zero ? zero4<T>() : v4_t<T>{(T)pf.q[u][0], (T)pf.q[u][1], (T)pf.q[u][2], (T)pf.q[u][3]};
    }
}

template <class T, int NX, int NU>
__device__ __forceinline__ void prefetch_stage(Prefetch<T, NX, NU> &pf, const StageSrc &s) {
    prefetch_mats(pf, s);
    prefetch_q(pf, s);
}

template <class T, int NX, int NU, bool RED, bool SOLVE>
__device__ __forceinline__ void commit_stage(MSmem<T, NX, NU, RED, SOLVE> &S, const Prefetch<T, NX, NU> &pf) {
    using PF = Prefetch<T, NX, NU>;
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < PF::NA; ++q) {
        const int e = tid + q * NT;
        if (e < NX * NX) S.A[e] = (T)pf.a_[q];
    }
#pragma unroll
    for (int q = 0; q < PF::NB; ++q) {
        const int e = tid + q * NT;
        if (e < NX * NU) S.B[e] = (T)pf.b_[q];
    }
    if (tid < NX) {
        S.av[tid] = (T)pf.av;
        S.lx[tid] = (T)pf.lx;
    }
    if (tid < NU) S.lw[tid] = (T)pf.lw;
    if (tid == 0) S.c = (T)pf.c;
}

// Orders one wavefront's LDS accesses (no workgroup barrier).
__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Value of lane N of this lane's row of 16 lanes (DPP row_newbcast; one
// 64-bit move for a double).
template <int N>
__device__ __forceinline__ double row_bcast(double v) {
    return __longlong_as_double(
        __builtin_amdgcn_update_dpp(0ll, __double_as_longlong(v), 0x150 + N, 0xF, 0xF, false));
}
template <int N>
__device__ __forceinline__ float row_bcast(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x150 + N, 0xF, 0xF, false));
}

__device__ __forceinline__ double rsq_est(double d) { return __builtin_amdgcn_rsq(d); }
__device__ __forceinline__ float rsq_est(float d) { return __builtin_amdgcn_rsqf(d); }

// Step K of chol_inv16: eliminate column K below the pivot in [G | I].
template <int K, class T>
__device__ __forceinline__ void chol16_step(T (&a)[8], int i, T &sdi, int &fail) {
    constexpr int kh = K >> 3, kc = K & 7;
    T d = bcast_lane(a[kc], 16 * kh + K);              // pivot d_K (wave-uniform)
    if (!(d > T(0)) || !__builtin_isfinite(d)) {
        fail = 1;
        d = T(1);
    }
    T is = rsq_est(d);
    is = is * (T(1.5) - T(0.5) * d * is * is);
    is = is * (T(1.5) - T(0.5) * d * is * is);
    if (i == K) sdi = is;
    const T f = __shfl(a[kc], 16 * kh + i, 64);       // entry (i, K) of this lane's row
    const T m = i > K ? f * (is * is) : T(0);           // rows above the pivot keep their values
#pragma unroll
    for (int c = 0; c < 8; ++c) a[c] -= m * row_bcast<K>(a[c]);
    if constexpr (K + 1 < 16) chol16_step<K + 1>(a, i, sdi, fail);
}

// chol_inv_wave for M = 16 with every lane of the wavefront at work: Gaussian
// elimination without pivoting on the 16 x 32 matrix [G | I] turns it into
// [D L_u' | L_u^{-1}] with G = L_u D L_u' (L_u unit lower triangular), i.e.
// the Cholesky factor L = L_u D^{1/2} and L^{-1} = D^{-1/2} L_u^{-1}, the
// same factorization and forward substitution as the row-per-lane sweep.
// Lane l holds row l % 16 of [G | I], columns 8 (l / 16) .. 8 (l / 16) + 7;
// the pivot row reaches the other lanes of each row of 16 by DPP, the pivot
// column by one bpermute, the pivot by readlane.
// The lane's row and column block are taken through an opaque copy: the
// compare masks formed from them (one per step) are the same in every stage,
// and the compiler would otherwise hoist all of them out of the caller's
// stage loop and keep them live in scalar registers (spilled to vector lanes).
template <class T>
__device__ __forceinline__ int chol_inv16(T *G, T *LiT) {
    int l = lane();
    asm volatile("" : "+v"(l));
    const int i = l & 15, h = l >> 4;
    T a[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const T g = G[i * 16 + ((8 * h + c) & 15)];
        a[c] = h < 2 ? g : (8 * (h - 2) + c == i ? T(1) : T(0));
    }
    int fail = 0;
    T sdi = T(0);
    chol16_step<0>(a, i, sdi, fail);
    if (h >= 2) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int j = 8 * (h - 2) + c;
            const T v = a[c] * sdi;
            G[i * 16 + j] = v;       // L^{-1}[i][j]
            LiT[j * 16 + i] = v;     // L^{-T}[j][i]
        }
    }
    return fail;
}

// Cholesky factorization G = L L' ("a factorization of G", Alg. 1) and the
// inverse L^{-1}, by one wavefront.  Lane i holds row i of G / L in
// registers; entries of other rows are broadcast with readlane, which places
// them in scalar registers, and the sweep is right-looking, so the dependency
// chain is one multiply-add per column.  The pivot's reciprocal square root
// comes from the hardware estimate refined by two Newton steps
// (r <- r (3 - d r^2) / 2, each doubling the correct bits), which replaces
// the much longer correctly-rounded square root and division sequences.
// L^{-1} is then formed column by column (lane c solves L x = e_c, again
// with readlane broadcasts).  On return G holds L^{-1} row-major and LiT
// holds L^{-T} row-major.  Returns nonzero
// (wave-uniform) if a pivot is not positive or not finite; a unit pivot is
// used in its place.
template <int M, class T>
__device__ __forceinline__ int chol_inv_wave(T *G, T *LiT) {
    static_assert(M <= 64, "one wavefront factors at most 64 rows");
    if constexpr (M == 16) return chol_inv16(G, LiT);
    const int ln = threadIdx.x & 63;
    T g[M];
#pragma unroll
    for (int j = 0; j < M; ++j) g[j] = (ln < M) ? G[ln * M + j] : T(0);
    int fail = 0;
    T invd = T(0);                       // 1 / L[ln][ln]
#pragma unroll
    for (int j = 0; j < M; ++j) {
        T d = bcast_lane(g[j], j);
        if (!(d > T(0)) || !__builtin_isfinite(d)) {
            fail = 1;
            d = T(1);
        }
        T is = __builtin_amdgcn_rsq(d);
        is = is * (T(1.5) - T(0.5) * d * is * is);
        is = is * (T(1.5) - T(0.5) * d * is * is);
        const T lij = (ln == j) ? d * is : g[j] * is;
        if (ln == j) invd = is;
        g[j] = lij;
#pragma unroll
        for (int k = j + 1; k < M; ++k) g[k] -= lij * bcast_lane(lij, k);
    }
    // lane c: column c of L^{-1}, from L x = e_c.  x starts at zero and its
    // c-th entry is set to 1 / L[c][c] at step c (where e_c would be scaled),
    // so no lane-dependent start vector is formed ahead of time (such a
    // vector, invariant across stages, is otherwise kept in scratch).
    // Column k of L is broadcast again here from a copy that the compiler
    // cannot see through, taken once x[k] is final: otherwise it would reuse
    // the factorization's broadcasts of the same entries, or hoist this
    // loop's broadcasts, and keep all of them live in scalar registers at
    // once (spilled to vector lanes and back).
    T x[M];
#pragma unroll
    for (int i = 0; i < M; ++i) x[i] = T(0);
#pragma unroll
    for (int k = 0; k < M; ++k) {
        T gk = g[k], dk = invd;
        asm volatile("" : "+v"(gk), "+v"(dk) : "v"(x[k]));
        const T ik = bcast_lane(dk, k);
        x[k] = (ln == k) ? ik : x[k] * ik;
#pragma unroll
        for (int i = k + 1; i < M; ++i) x[i] -= bcast_lane(gk, i) * x[k];
    }
    if (ln < M) {
#pragma unroll
        for (int i = 0; i < M; ++i) {
            G[i * M + ln] = x[i];        // L^{-1}[i][ln]
            LiT[ln * M + i] = x[i];      // L^{-T}[ln][i]
        }
    }
    return fail;
}

// 32 x 32 version of chol_inv_wave by 2 x 2 blocks of 16, run by the whole
// workgroup (every thread must call it):
//   L11 = chol(G11), L21 = G21 L11^{-T}, L22 = chol(G22 - L21 L21'),
//   L^{-1} = [L11^{-1}, 0; -L22^{-1} L21 L11^{-1}, L22^{-1}].
// The two 16 x 16 factorizations are chol_inv_wave<16> on wave 0 (a shorter
// dependency chain and a quarter of the registers of the 32 x 32 sweep); the
// block products are single 16x16 matrix-core tiles.  `side` is run by
// waves 1-3 while wave 0 factors the first block.  LiT and G serve as
// scratch (four 16 x 16 blocks in LiT, three in G).  On return G holds
// L^{-1} and LiT holds L^{-T}, row-major; *bad is set if a pivot failed.
template <class T, class Side>
__device__ __forceinline__ void chol_inv_block32(T *G, T *LiT, int *bad, Side side) {
    constexpr int M = 32, H = 16;
    const int tid = threadIdx.x, w = wave(), l = lane();
    T *T0 = LiT, *T1 = LiT + 256, *T2 = LiT + 512, *T3 = LiT + 768;   // L11^-1, L11^-T, L21, G22 - L21 L21'
    T *Gt = G, *Gm = G + 256, *Gc = G + 512;                         // L22^-T, L21 L11^-1, C
    for (int e = tid; e < H * H; e += NT) T0[e] = G[(e / H) * M + e % H];
    lds_sync();
    if (w == 0) {
        int f = chol_inv_wave<H>(T0, T1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // L21 = G21 L11^{-T}
        v4_t<T> acc = mma<H, false, false>(zero4<T>(), G + H * M, M, T1, H, 0, 0);
        tile_for<T>(0, 0, [&](int r, int i, int j) { T2[i * H + j] = acc[r]; });
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // Schur complement G22 - L21 L21'
        acc = mma<H, false, true>(zero4<T>(), T2, H, T2, H, 0, 0);
        tile_for<T>(0, 0, [&](int r, int i, int j) { T3[i * H + j] = G[(H + i) * M + H + j] - acc[r]; });
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        f |= chol_inv_wave<H>(T3, Gt);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // C = -L22^{-1} (L21 L11^{-1})
        acc = mma<H, false, false>(zero4<T>(), T2, H, T0, H, 0, 0);
        tile_for<T>(0, 0, [&](int r, int i, int j) { Gm[i * H + j] = acc[r]; });
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        acc = mma<H, false, false>(zero4<T>(), T3, H, Gm, H, 0, 0);
        tile_for<T>(0, 0, [&](int r, int i, int j) { Gc[i * H + j] = -acc[r]; });
        if (f && l == 0) *bad = 1;
    } else {
        side();
    }
    lds_sync();
    constexpr int R = M * M / NT;
    T li[R], lt[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int e = tid + q * NT, i = e / M, j = e % M;
        const int bi = i & (H - 1), bj = j & (H - 1);
        if (i < H) {
            li[q] = j < H ? T0[bi * H + bj] : T(0);
            lt[q] = j < H ? T1[bi * H + bj] : Gc[bj * H + bi];
        } else {
            li[q] = j < H ? Gc[bi * H + bj] : T3[bi * H + bj];
            lt[q] = j < H ? T(0) : Gt[bi * H + bj];
        }
    }
    lds_sync();
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int e = tid + q * NT;
        G[e] = li[q];
        LiT[e] = lt[q];
    }
}

// Wave-level sum over the 64 lanes (result in every lane).

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ====================================================== one Riccati pass
// Backward pass over `count` stages (local s = count-1 .. 0).  Starting
// state (P, Psi, cbar; and V = I, v = 0, Q_w_hat = 0 for RED) must be in LDS.
//   RED   : Alg. 4 (reduction with the preliminary terminal P = 0)
//   SOLVE : Alg. 1-2 forming K, k; out.K / out.P / out.Psi / out.k receive
//           K_{t+1}, P_t, Psi_t, k_{t+1} of stage s from the lanes that
//           computed them; pre(s) sees P_{t+1}, Psi_{t+1}, cbar_{t+1}
//   neither: elimination of a subproblem with known terminal (Alg. 1-2)
template <class T, int NX, int NU, bool RED, bool SOLVE, class Get, class Pre, class Out>
__device__ void mfma_pass(MSmem<T, NX, NU, RED, SOLVE> &S, Get get, int count, int32_t *info, int inst,
                          int stage_base, int fail_code, Pre pre, Out out) {
    static_assert(NX % 16 == 0 && NU % 16 == 0, "MFMA path needs multiples of 16");
    static_assert(NX <= 64 && NU <= 64, "per-wave vector roles assume NX, NU <= 64");
    constexpr int NW = NX + NU, TX = NX / 16, TU = NU / 16;
    constexpr bool VEC = Out::VEC, KFORM = SOLVE || Out::KF, PEMIT = SOLVE || Out::PF;
    constexpr bool LTFORM = RED && Out::LTF, PSEMIT = SOLVE || Out::PSF, KVEC = VEC && (SOLVE || Out::KVF);
    const int tid = threadIdx.x, w = wave(), l = lane();
    count = uni(count);
    Prefetch<T, NX, NU> pf;
    v4_t<T> qt[Tiles<NX, NU>::PER_WAVE];
    if (tid == 0) S.bad = 0;
    if (count > 0) {
        prefetch_stage<T, NX, NU>(pf, get(count - 1));
        wait_global();
        commit_stage(S, pf);
        take_q(qt, pf);
    }
    lds_sync();
    // The next stage's inputs (A, B, stage vectors and the Q tiles) are
    // loaded into registers at the start of a stage and committed at the
    // start of phase E (nothing in phase E reads A, B or the stage vectors),
    // after an explicit wait for them and before phase E issues its global
    // stores.  The loads have the stage's first phases to arrive.
    for (int s = count - 1; s >= 0; --s) {
        // stage s inputs: A, B, a, lx, lw, c in LDS; Qx/Qxw'/Qw tiles in qt
        // the next stage's source (pointers and c), formed once per stage
        const StageSrc nxt = s > 0 ? get(s - 1) : StageSrc{};
        if (s > 0) prefetch_stage<T, NX, NU>(pf, nxt);
        pre(s, S);
        using TT = Tiles<NX, NU>;
        v4_t<T> fkeep[TT::PER_WAVE_F];      // F tiles of this wave (merged phase)
        if constexpr (TT::FAST) {
            // ---- merged phases A-C (n_u = 16): wave 0: W_B = P B, G = Qw + B'W_B, L^{-1};
            //      wave 1 + tj: W_A column tj, F and H' tiles of column tj;
            //      wave RW (RED): B'V, A'V, V'a; wave 3: P a, Psi - P a, cbar, g_x, g_w
            constexpr int RW = TX == 1 ? 2 : 3;
            if (w == 0) {
#pragma unroll
                for (int ti = 0; ti < TX; ++ti) {
                    v4_t<T> acc = mma<NX, true, false>(zero4<T>(), S.P, NX, S.B, NU, ti, 0);
                    tile_for<T>(ti, 0, [&](int r, int i, int j) { S.W[i * NW + NX + j] = acc[r]; });
                }
                wave_fence();
                {
                    constexpr int tg = TT::TF + TT::TH;
                    v4_t<T> acc = mma<NX, true, false>(qt[TT::slot(tg)], S.B, NU, S.W + NX, NW, 0, 0);
                    tile_for<T>(0, 0, [&](int r, int i, int j) { put_sym(S.G, NU, 0, 0, i, j, acc[r]); });
                }
                wave_fence();
                const int f = chol_inv_wave<NU>(S.G, S.LiT);
                if (f && l == 0) S.bad = 1;
            } else if (w <= TX) {
                const int tj = w - 1;
#pragma unroll
                for (int ti = 0; ti < TX; ++ti) {
                    v4_t<T> acc = mma<NX, true, false>(zero4<T>(), S.P, NX, S.A, NX, ti, tj);
                    tile_for<T>(ti, tj, [&](int r, int i, int j) { S.W[i * NW + j] = acc[r]; });
                }
                wave_fence();
#pragma unroll
                for (int t = 0; t < TT::TF + TT::TH; ++t) {
                    if (TT::owner(t) != w) continue;
                    int kind, ti, tjj;
                    phaseB_tile<NX, NU>(t, kind, ti, tjj);
                    if (kind == 0) {
                        fkeep[TT::fslot(t)] = mma<NX, true, false>(qt[TT::slot(t)], S.A, NX, S.W, NW, ti, tjj);
                    } else {
                        v4_t<T> acc = mma<NX, true, false>(qt[TT::slot(t)], S.B, NU, S.W, NW, ti, tjj);
                        tile_for<T>(ti, tjj, [&](int r, int i, int j) { S.HT[i * NX + j] = acc[r]; });
                    }
                }
            }
            if constexpr (RED) {
                if (w == RW) {
#pragma unroll
                    for (int tj = 0; tj < TX; ++tj) {
                        v4_t<T> acc = mma<NX, true, false>(zero4<T>(), S.B, NU, S.V, NX, 0, tj);
                        tile_for<T>(0, tj, [&](int r, int i, int j) { S.BV[i * NX + j] = acc[r]; });
                    }
#pragma unroll
                    for (int t = 0; t < TX * TX; ++t) {
                        const int ti = t / TX, tj = t % TX;
                        v4_t<T> acc = mma<NX, true, false>(zero4<T>(), S.A, NX, S.V, NX, ti, tj);
                        tile_for<T>(ti, tj, [&](int r, int i, int j) { S.AV[i * NX + j] = acc[r]; });
                    }
                    if (VEC && l < NX) {
                        T acc = T(0);
#pragma unroll 8
                        for (int k = 0; k < NX; ++k) acc += S.V[k * NX + l] * S.av[k];
                        S.Vta[l] = acc;
                    }
                }
            }
            // Vector lines: pt = Psi - P a, cbar, g_x = A'pt - l_x, g_w = B'pt - l_w.
            // In the reduction with n_x = 32, wave 3 has the B'V and A'V
            // tiles, so waves 1 and 2 (the lighter matrix roles) take the
            // vector lines, each forming pt itself: wave 1 also cbar and g_x,
            // wave 2 g_w.  Otherwise wave 3 does all of them.
            constexpr int VA = (RED && TX == 2) ? 1 : 3, VB = (RED && TX == 2) ? 2 : 3;
            if (VEC && (w == VA || w == VB)) {
                T *pt = w == VA ? S.pt : S.pt2;
                T part = T(0);
                if (l < NX) {
                    T pa = T(0);
#pragma unroll 8
                    for (int k = 0; k < NX; ++k) pa += S.P[k * NX + l] * S.av[k];
                    pt[l] = S.Psi[l] - pa;
                    part = S.av[l] * (T(0.5) * pa - S.Psi[l]);
                }
                if (w == VA) {
                    // cbar += 1/2 a'Pa - Psi'a + c (Alg. 2, with P_{t+1}, Psi_{t+1})
                    part = wave_sum(part);
                    if (l == 0) S.cbar += part + S.c;
                }
                wave_fence();
                if (w == VA && l < NX) {
                    T acc = -S.lx[l];
#pragma unroll 8
                    for (int k = 0; k < NX; ++k) acc += S.A[k * NX + l] * pt[k];
                    S.gx[l] = acc;
                }
                const int iw = VA == VB ? l - NX : l;
                if (w == VB && iw >= 0 && iw < NU) {
                    T acc = -S.lw[iw];
#pragma unroll 8
                    for (int k = 0; k < NX; ++k) acc += S.B[k * NU + iw] * pt[k];
                    S.gw[iw] = acc;
                }
            }
        } else {
            // ---- phase A: W = P[A B], (RED) B'V; P a, Psi - P a, (RED) V'a
            {
                constexpr int TW = TX * (TX + TU), TBV = RED ? TU * TX : 0;
                for (int t = w; t < TW + TBV; t += 4) {
                    v4_t<T> acc = zero4<T>();
                    if (t < TW) {
                        const int ti = t / (TX + TU), tj = t % (TX + TU);
                        if (tj < TX)
                            acc = mma<NX, true, false>(acc, S.P, NX, S.A, NX, ti, tj);
                        else
                            acc = mma<NX, true, false>(acc, S.P, NX, S.B, NU, ti, tj - TX);
                        tile_for<T>(ti, tj, [&](int r, int i, int j) { S.W[i * NW + j] = acc[r]; });
                    } else if constexpr (RED) {
                        const int u = t - TW, ti = u / TX, tj = u % TX;
                        acc = mma<NX, true, false>(acc, S.B, NU, S.V, NX, ti, tj);
                        tile_for<T>(ti, tj, [&](int r, int i, int j) { S.BV[i * NX + j] = acc[r]; });
                    }
                }
                if (VEC && w == 3) {
                    T part = T(0);
                    if (l < NX) {
                        T pa = T(0);
    #pragma unroll 8
                        for (int k = 0; k < NX; ++k) pa += S.P[k * NX + l] * S.av[k];
                        S.pt[l] = S.Psi[l] - pa;
                        part = S.av[l] * (T(0.5) * pa - S.Psi[l]);
                    }
                    // cbar += 1/2 a'Pa - Psi'a + c (Alg. 2, with P_{t+1}, Psi_{t+1})
                    part = wave_sum(part);
                    if (l == 0) S.cbar += part + S.c;
                } else if (VEC && RED && tid >= 128 && tid < 128 + NX) {
                    const int i = tid - 128;
                    T acc = T(0);
    #pragma unroll 8
                    for (int k = 0; k < NX; ++k) acc += S.V[k * NX + i] * S.av[k];
                    S.Vta[i] = acc;
                }
            }
            lds_sync();
            // ---- phase B: F = Qx + A'W_A (lower), H' = Qxw' + B'W_A, G = Qw + B'W_B (lower)
            {
                using PF = Tiles<NX, NU>;
    #pragma unroll
                for (int u = 0; u < PF::PER_WAVE; ++u) {
                    const int t = w + 4 * u;
                    if (t < PF::TILES) {
                        int kind, ti, tj;
                        phaseB_tile<NX, NU>(t, kind, ti, tj);
                        v4_t<T> acc = qt[u];
                        if (kind == 0) {
                            acc = mma<NX, true, false>(acc, S.A, NX, S.W, NW, ti, tj);
                            tile_for<T>(ti, tj, [&](int r, int i, int j) { put_sym(S.F(), NX, ti, tj, i, j, acc[r]); });
                        } else if (kind == 1) {
                            acc = mma<NX, true, false>(acc, S.B, NU, S.W, NW, ti, tj);
                            tile_for<T>(ti, tj, [&](int r, int i, int j) { S.HT[i * NX + j] = acc[r]; });
                        } else {
                            acc = mma<NX, true, false>(acc, S.B, NU, S.W + NX, NW, ti, tj);
                            tile_for<T>(ti, tj, [&](int r, int i, int j) { put_sym(S.G, NU, ti, tj, i, j, acc[r]); });
                        }
                    }
                }
                if (VEC && tid >= 192 && tid < 192 + NX) {
                    const int i = tid - 192;
                    T acc = -S.lx[i];
    #pragma unroll 8
                    for (int k = 0; k < NX; ++k) acc += S.A[k * NX + i] * S.pt[k];
                    S.gx[i] = acc;
                } else if (VEC && tid >= 128 && tid < 128 + NU) {
                    const int i = tid - 128;
                    T acc = -S.lw[i];
    #pragma unroll 8
                    for (int k = 0; k < NX; ++k) acc += S.B[k * NU + i] * S.pt[k];
                    S.gw[i] = acc;
                }
            }
            lds_sync();
            // ---- phase C: factor and invert G (wave 0); (RED) A'V into W (waves 1-3)
            auto av_tiles = [&]() {
                if constexpr (RED) {
                    for (int t = w - 1; t < TX * TX; t += 3) {
                        const int ti = t / TX, tj = t % TX;
                        v4_t<T> acc = mma<NX, true, false>(zero4<T>(), S.A, NX, S.V, NX, ti, tj);
                        tile_for<T>(ti, tj, [&](int r, int i, int j) { S.W[i * NX + j] = acc[r]; });
                    }
                }
            };
            if constexpr (NU == 32) {
                chol_inv_block32(S.G, S.LiT, &S.bad, av_tiles);
            } else {
                if (w == 0) {
                    const int f = chol_inv_wave<NU>(S.G, S.LiT);
                    if (f && l == 0) S.bad = 1;
                } else {
                    av_tiles();
                }
            }
        }
        lds_sync();
        if (tid == 0 && S.bad) {
            record_failure(info, inst, fail_code, stage_base < 0 ? -1 : stage_base + s);
            S.bad = 0;
        }
        // ---- phase D: Y = L^{-1} H', (RED) X = L^{-1} B'V, z = L^{-1} g_w
        {
            constexpr int TY = TU * TX, TXX = RED ? TU * TX : 0;
            for (int t = w; t < TY + TXX; t += 4) {
                const int u = t < TY ? t : t - TY, ti = u / TX, tj = u % TX;
                if (t < TY) {
                    v4_t<T> acc = mma<NU, true, false>(zero4<T>(), S.LiT, NU, S.HT, NX, ti, tj);
                    tile_for<T>(ti, tj, [&](int r, int i, int j) { S.Y()[i * NX + j] = acc[r]; });
                } else if constexpr (RED) {
                    v4_t<T> acc = mma<NU, true, false>(zero4<T>(), S.LiT, NU, S.BV, NX, ti, tj);
                    tile_for<T>(ti, tj, [&](int r, int i, int j) { S.X[i * NX + j] = acc[r]; });
                }
            }
            if (VEC && tid >= 192 && tid < 192 + NU) {
                const int i = tid - 192;
                T acc = T(0);
#pragma unroll
                for (int k = 0; k < NU; ++k) acc += S.LiT[k * NU + i] * S.gw[k];
                S.z[i] = acc;
            }
        }
        lds_sync();
        // ---- phase E: P = F - Y'Y, (RED) Q_w_hat += X'X, V = A'V - Y'X,
        //      (SOLVE) K = -L^{-T} Y, k = L^{-T} z;
        //      Psi = g_x - Y'z, (RED) v += V'a + X'z, cbar -= z'z/2
        {
            // the wait is on every path: where it is skipped, the compiler
            // takes the prefetch loads as still outstanding at the next
            // stage and waits for them (and for every store behind them)
            // when their registers are reused
            wait_global();
            if (s > 0) {
                commit_stage(S, pf);
                take_q(qt, pf);
            }
            constexpr int TL = TX * (TX + 1) / 2, TQ = RED ? TL : 0, TV = RED ? TX * TX : 0,
                          TK = KFORM ? TU * TX : 0, TLT = LTFORM ? TU * TX : 0;
            if constexpr (TT::FAST) {
                // P = F - Y'Y on the waves that hold the F tiles
#pragma unroll
                for (int t = 0; t < TL; ++t) {
                    if (TT::owner(t) != w) continue;
                    int ti, tj;
                    lower_tile(t, ti, tj);
                    v4_t<T> acc = mma<NU, true, false>(zero4<T>(), S.Y(), NX, S.Y(), NX, ti, tj);
                    const v4_t<T> fv = fkeep[TT::fslot(t)];
                    tile_for<T>(ti, tj, [&](int r, int i, int j) {
                        if (ti != tj || i >= j) {
                            const T v = fv[r] - acc[r];
                            S.P[i * NX + j] = v;
                            S.P[j * NX + i] = v;
                        }
                    });          // the P_t record is written from LDS after the stage
                }
            }
            // the other tiles in wave order 0, 3, 2, 1 when the F owners
            // already have the P tiles
            const int first = TT::FAST ? TL + ((4 - w) & 3) : w;
            for (int t = first; t < TL + TQ + TV + TK + TLT; t += 4) {
                if (t < TL) {
                    int ti, tj;
                    lower_tile(t, ti, tj);
                    v4_t<T> acc = mma<NU, true, false>(zero4<T>(), S.Y(), NX, S.Y(), NX, ti, tj);
                    tile_for<T>(ti, tj, [&](int r, int i, int j) {
                        if (ti != tj || i >= j) {
                            const T v = S.F()[i * NX + j] - acc[r];
                            S.P[i * NX + j] = v;
                            S.P[j * NX + i] = v;
                            if constexpr (PEMIT) {
                                out.P(s, i, j, v);
                                if (i != j) out.P(s, j, i, v);
                            }
                        }
                    });
                } else if (t < TL + TQ) {
                    if constexpr (RED) {
                        int ti, tj;
                        lower_tile(t - TL, ti, tj);
                        v4_t<T> acc = mma<NU, true, false>(zero4<T>(), S.X, NX, S.X, NX, ti, tj);
                        tile_for<T>(ti, tj, [&](int r, int i, int j) {
                            put_sym(S.Qh, NX, ti, tj, i, j, S.Qh[i * NX + j] + acc[r]);
                        });
                    }
                } else if (t < TL + TQ + TV) {
                    if constexpr (RED) {
                        const int u = t - TL - TQ, ti = u / TX, tj = u % TX;
                        v4_t<T> acc = mma<NU, true, false>(zero4<T>(), S.Y(), NX, S.X, NX, ti, tj);
                        const T *av = TT::FAST ? S.AV : S.W;       // A'V
                        tile_for<T>(ti, tj, [&](int r, int i, int j) {
                            const T v = av[i * NX + j] - acc[r];
                            S.V[i * NX + j] = v;
                            if constexpr (Out::VF) out.V(s, i, j, v);
                        });
                    }
                } else if (t < TL + TQ + TV + TK) {
                    if constexpr (KFORM) {
                        const int u = t - TL - TQ - TV, ti = u / TX, tj = u % TX;
                        v4_t<T> acc = mma<NU, true, false>(zero4<T>(), S.G, NU, S.Y(), NX, ti, tj);
                        tile_for<T>(ti, tj, [&](int r, int i, int j) { out.K(s, i, j, -acc[r]); });
                    }
                } else {
                    if constexpr (LTFORM) {
                        const int u = t - TL - TQ - TV - TK, ti = u / TX, tj = u % TX;
                        v4_t<T> acc = mma<NU, true, false>(zero4<T>(), S.G, NU, S.X, NX, ti, tj);
                        tile_for<T>(ti, tj, [&](int r, int i, int j) { out.Lt(s, i, j, -acc[r]); });
                    }
                }
            }
            if constexpr (Out::LF) out.L(s, S.G);
            if (VEC && tid >= 192 && tid < 192 + NX) {
                const int i = tid - 192;
                T acc = S.gx[i];
#pragma unroll
                for (int r = 0; r < NU; ++r) acc -= S.Y()[r * NX + i] * S.z[r];
                S.Psi[i] = acc;
                if constexpr (PSEMIT) out.Psi(s, i, acc);
            } else if (VEC && RED && tid >= 128 && tid < 128 + NX) {
                const int i = tid - 128;
                T acc = S.Vta[i];
#pragma unroll
                for (int r = 0; r < NU; ++r) acc += S.X[r * NX + i] * S.z[r];
                S.v[i] += acc;
            } else if (KVEC && tid < NU) {
                // k_{t+1} = L^{-T} z (wave 0 has no other vector work here)
                const int i = tid;
                T acc = T(0);
#pragma unroll
                for (int r = 0; r < NU; ++r) acc += S.G[r * NU + i] * S.z[r];
                S.kk[i] = acc;
                out.k(s, i, acc);
            } else if (VEC && tid >= 64 && tid < 128) {
                const T zz = wave_sum(l < NU ? S.z[l] * S.z[l] : T(0));
                if (l == 0) S.cbar -= T(0.5) * zz;
            }
        }
        lds_sync();
        if constexpr (PEMIT && TT::FAST) {
            // P_t record row by row from LDS: consecutive threads store
            // consecutive elements, and no per-tile store offsets stay live
            // across the stage (S.P is next written in the next phase E)
            for (int e = tid; e < NX * NX; e += NT) out.P(s, e / NX, e % NX, S.P[e]);
        }
    }
}

}  // namespace mf
}  // namespace rs
