// Device-side building blocks of the parallel Riccati solver for gfx950:
// small LDS-resident matrix products, a wavefront Cholesky factorization with
// cross-lane broadcasts, column-parallel triangular solves, and the per-stage
// Riccati recursion in its three uses:
//
//   reduce (Alg. 4)        subproblem with unknown terminal, P = 0 start,
//                          yields A_hat, Q_w_hat (= B_hat), a_hat, Q_x_hat, l_x_hat, c_hat
//   eliminate (Sec. 4.2)   last subproblem with known terminal: Alg. 1-2 only,
//                          yields the terminal cost it passes up
//   solve (Alg. 1-3)       subproblem with known terminal and initial state,
//                          Alg. 6's per-node solve
//
// One workgroup of NT threads owns one subproblem; its stages are processed
// backwards one at a time with every operand in LDS.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rs_types.hpp"

namespace rs {

constexpr int NT = 256;          // threads per workgroup (4 wavefronts)

// ------------------------------------------------------------------ scalars
__device__ __forceinline__ double bcast_lane(double v, int lane) {
    int64_t b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(uint32_t)(b & 0xffffffffll), lane);
    int hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)b >> 32), lane);
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ __forceinline__ float bcast_lane(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
// Wave-uniform copy of an integer that is the same in every lane.  Loop
// bounds and branch conditions around barriers go through this so that the
// compiler sees uniform control flow and keeps every barrier in lock-step.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Instance excluded from this call (its descriptor carries PROB_SKIP).
__device__ __forceinline__ bool inst_skipped(const DevProb *probs, int inst) {
    return (uni(probs[inst].flags) & PROB_SKIP) != 0;
}

// Workgroup barrier that orders LDS only.  __syncthreads() also orders
// global memory, which makes every wave wait for all of its outstanding
// global loads and stores (the next stage's prefetch, the records just
// written) at each barrier; the passes only exchange data through LDS
// between their phases, so their barriers leave global traffic in flight.
__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Load through a global-address-space pointer.  Problem data are reached
// through pointers read from descriptors, which the compiler would access
// with flat instructions; flat loads also count as LDS operations, so every
// LDS wait before a barrier would then wait for them too.  Global loads
// leave the prefetched data in flight across the barriers.
template <class T>
__device__ __forceinline__ T gload(const T *p) {
    typedef const __attribute__((address_space(1))) T *gptr;
    return *(gptr)(p);
}

__device__ __forceinline__ double rs_sqrt(double v) { return sqrt(v); }
__device__ __forceinline__ float rs_sqrt(float v) { return sqrtf(v); }

// -------------------------------------------------- small matrix products
// out(i, j, acc) with acc = sum_k opA(i,k) opB(k,j) for i < M, j < N, split
// over threads [tid0, tid0 + nthr).  opA(i,k) = TA ? A[k*lda+i] : A[i*lda+k],
// opB(k,j) = TB ? B[j*ldb+k] : B[k*ldb+j].  Each thread owns 2x2 output tiles
// when M and N are even (two LDS reads per two FMAs), else single outputs.
template <int M, int N, int K, bool TA, bool TB, class T, class Out>
__device__ __forceinline__ void mm(const T *__restrict__ A, int lda, const T *__restrict__ B,
                                   int ldb, int tid, int nthr, Out out) {
    if constexpr (M % 2 == 0 && N % 2 == 0) {
        constexpr int TN = N / 2, TILES = (M / 2) * (N / 2);
        for (int idx = tid; idx < TILES; idx += nthr) {
            const int i = 2 * (idx / TN), j = 2 * (idx % TN);
            T c00 = 0, c01 = 0, c10 = 0, c11 = 0;
#pragma unroll 4
            for (int k = 0; k < K; ++k) {
                const T a0 = TA ? A[k * lda + i] : A[i * lda + k];
                const T a1 = TA ? A[k * lda + i + 1] : A[(i + 1) * lda + k];
                const T b0 = TB ? B[j * ldb + k] : B[k * ldb + j];
                const T b1 = TB ? B[(j + 1) * ldb + k] : B[k * ldb + j + 1];
                c00 += a0 * b0;
                c01 += a0 * b1;
                c10 += a1 * b0;
                c11 += a1 * b1;
            }
            out(i, j, c00);
            out(i, j + 1, c01);
            out(i + 1, j, c10);
            out(i + 1, j + 1, c11);
        }
    } else {
        for (int idx = tid; idx < M * N; idx += nthr) {
            const int i = idx / N, j = idx % N;
            T acc = 0;
#pragma unroll 4
            for (int k = 0; k < K; ++k)
                acc += (TA ? A[k * lda + i] : A[i * lda + k]) * (TB ? B[j * ldb + k] : B[k * ldb + j]);
            out(i, j, acc);
        }
    }
}

// y(i) = sum_k opA(i,k) x[k], i < M, threads [tid0, tid0+nthr)
template <int M, int K, bool TA, class T, class Out>
__device__ __forceinline__ void mv(const T *__restrict__ A, int lda, const T *__restrict__ x, int tid,
                                   int nthr, Out out) {
    for (int i = tid; i < M; i += nthr) {
        T acc = 0;
#pragma unroll 4
        for (int k = 0; k < K; ++k) acc += (TA ? A[k * lda + i] : A[i * lda + k]) * x[k];
        out(i, acc);
    }
}

// ---------------------------------------------------- Cholesky, one wave
// G (M x M row-major, LDS) is replaced by its lower Cholesky factor L
// (G = L L', "a factorization of G", Alg. 1); dinv[i] = 1 / L[i][i].
// Lane i holds row i in registers; column j is broadcast with readlane.
// Must be called by all 64 lanes of one wavefront.  Returns nonzero (wave
// uniform) if a pivot is not positive or not finite; the factorization then
// continues with a unit pivot so that no NaN reaches later stages.
template <int M, class T>
__device__ __forceinline__ int chol_wave(T *G, T *dinv) {
    static_assert(M <= 64, "one wavefront factors at most 64 rows");
    const int lane = threadIdx.x & 63;
    T g[M];
#pragma unroll
    for (int j = 0; j < M; ++j) g[j] = (lane < M) ? G[lane * M + j] : T(0);
    int fail = 0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        T d = bcast_lane(g[j], j);
        if (!(d > T(0)) || !(d < T(1e300))) {
            fail = 1;
            d = T(1);
        }
        const T s = rs_sqrt(d);
        const T is = T(1) / s;
        const T lij = (lane == j) ? s : g[j] * is;
        g[j] = lij;
#pragma unroll
        for (int k = j + 1; k < M; ++k) {
            const T lkj = bcast_lane(lij, k);
            g[k] -= lij * lkj;
        }
    }
    if (lane < M) {
#pragma unroll
        for (int j = 0; j < M; ++j) G[lane * M + j] = (j <= lane) ? g[j] : T(0);
        dinv[lane] = T(1) / g[lane];
    }
    return fail;
}

// Forward substitution L y = b for one column held by the calling thread.
template <int M, class T>
__device__ __forceinline__ void trsv_l(const T *__restrict__ L, const T *__restrict__ dinv, T (&y)[M]) {
#pragma unroll
    for (int i = 0; i < M; ++i) {
        T s = y[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i * M + k] * y[k];
        y[i] = s * dinv[i];
    }
}
// Backward substitution L' y = b for one column held by the calling thread.
template <int M, class T>
__device__ __forceinline__ void trsv_lt(const T *__restrict__ L, const T *__restrict__ dinv, T (&y)[M]) {
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
        T s = y[i];
#pragma unroll
        for (int k = i + 1; k < M; ++k) s -= L[k * M + i] * y[k];
        y[i] = s * dinv[i];
    }
}

// ------------------------------------------------------------ stage data
// Pointers to one stage's data in global memory (FP64).  Leaves point into
// the caller's problem arrays; master stages point into slots, where
// Q_xw = 0, l_w = 0 and B = Q_w = Q_w_hat (Theorem 1 with the T-transform).
struct StageSrc {
    const double *Qx, *Qw, *Qxw, *A, *B, *a, *lx, *lw;
    double c;
    const double *cp;      // where c is read from (nullptr: c = 0), for prefetching passes
};

// Problem descriptor copied once into wave-uniform registers.  Reading it
// through the global-memory reference at every stage would re-issue a chain of
// dependent loads (the compiler cannot prove the descriptor unchanged across
// the kernel's own global stores).
__device__ __forceinline__ const double *uni_ptr(const double *q) {
    const uint64_t v = (uint64_t)q;
    const uint32_t lo = (uint32_t)uni((int)(uint32_t)(v & 0xffffffffu)), hi = (uint32_t)uni((int)(uint32_t)(v >> 32));
    return (const double *)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int64_t uni64(int64_t v) {
    const uint32_t lo = (uint32_t)uni((int)(uint32_t)((uint64_t)v & 0xffffffffu)),
                   hi = (uint32_t)uni((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ DevProb load_prob(const DevProb *tab, int i) {
    const DevProb r = tab[i];
    DevProb u;
    u.Qx = uni_ptr(r.Qx);
    u.Qw = uni_ptr(r.Qw);
    u.Qxw = uni_ptr(r.Qxw);
    u.A = uni_ptr(r.A);
    u.B = uni_ptr(r.B);
    u.QxN = uni_ptr(r.QxN);
    u.x0 = uni_ptr(r.x0);
    u.a = uni_ptr(r.a);
    u.lx = uni_ptr(r.lx);
    u.lw = uni_ptr(r.lw);
    u.c = uni_ptr(r.c);
    u.lN = uni_ptr(r.lN);
    u.cN = uni_ptr(r.cN);
    u.x = const_cast<double *>(uni_ptr(r.x));
    u.w = const_cast<double *>(uni_ptr(r.w));
    u.lam = const_cast<double *>(uni_ptr(r.lam));
    u.obj = const_cast<double *>(uni_ptr(r.obj));
    u.sQx = uni64(r.sQx);
    u.sQw = uni64(r.sQw);
    u.sQxw = uni64(r.sQxw);
    u.sA = uni64(r.sA);
    u.sB = uni64(r.sB);
    u.sa = uni64(r.sa);
    u.slx = uni64(r.slx);
    u.slw = uni64(r.slw);
    u.sc = uni64(r.sc);
    u.nx = uni(r.nx);
    u.nu = uni(r.nu);
    u.N = uni(r.N);
    u.flags = uni(r.flags);
    return u;
}

__device__ __forceinline__ StageSrc prob_stage(const DevProb &p, int t) {
    StageSrc s;
    s.Qx = p.Qx + (int64_t)t * p.sQx;
    s.Qw = p.Qw + (int64_t)t * p.sQw;
    s.Qxw = p.Qxw ? p.Qxw + (int64_t)t * p.sQxw : nullptr;
    s.A = p.A + (int64_t)t * p.sA;
    s.B = p.B + (int64_t)t * p.sB;
    s.a = p.a ? p.a + (int64_t)t * p.sa : nullptr;
    s.lx = p.lx ? p.lx + (int64_t)t * p.slx : nullptr;
    s.lw = p.lw ? p.lw + (int64_t)t * p.slw : nullptr;
    s.cp = p.c ? p.c + (int64_t)t * p.sc : nullptr;
    s.c = s.cp ? gload(s.cp) : 0.0;
    return s;
}

// A master stage (Sec. 4.3, eq. red_mpc_problem) read from the M1 message
// in its slot: B = Q_w = Q_w_hat (the form of eq. Qh_Bh_alternative_def), or,
// with `ident` (an n x n identity), B = the rank-revealing factor written in
// the Q_w_hat place and Q_w = I (see rank_reveal).
__device__ __forceinline__ StageSrc slot_stage(const double *slot, int n, const double *ident) {
    const SlotLayout L{n};
    StageSrc s;
    s.Qx = slot + L.Qx();
    s.Qw = ident ? ident : slot + L.Qw();
    s.Qxw = nullptr;
    s.A = slot + L.A();
    s.B = slot + L.Qw();
    s.a = slot + L.a();
    s.lx = slot + L.lx();
    s.lw = nullptr;
    s.cp = slot + L.c();
    s.c = *s.cp;
    return s;
}

// Rank-revealing form of a reduced subproblem (Sec. 4.2, eqs. Bh_def and
// Gh_Hh_def).  The reduction (Alg. 4) leaves M = S Qbar^{-1} S' in `M`
// (n x n, row-major, positive semidefinite of rank n_uo = rank(S')).  This
// factors it by Cholesky with diagonal pivoting, M ~= B B' with column c of
// B the c-th pivot column, and stops once the largest remaining diagonal
// entry is at most n eps max_i M_ii (the usual stopping rule of pivoted
// Cholesky; the remaining Schur complement, positive semidefinite, is then
// below that bound entrywise).  Columns from the rank on are zero.
// A master stage with input matrix B and input weight I has
// B I^{-1} B' = M, as does the stage of the U_1 basis
// (B_hat Q_w_hat^{-1} B_hat' = S Qbar^{-1} S'); a master stage enters the
// master problem only through that product (minimising its input cost for a
// given state step), so both master problems have the same states and
// costates, and G = I + B'PB of the stage is positive definite even when
// N_s n_u < n_x or the subinterval's inputs leave state directions
// unreached.  Zero columns are inputs that move nothing and stay 0.
// B goes to out (and cache if given), row-major n x n; M is overwritten.
// Every thread of the workgroup calls; thread i owns row i
// (n <= blockDim.x, n <= 128, at most 16 wavefronts).
template <class T>
__device__ __attribute__((noinline)) void rank_reveal(T *M, int n, double eps, double *out, double *cache) {
    __shared__ double s_val[2][16];
    __shared__ int s_idx[2][16];
    const int tid = threadIdx.x, nw = (int)(blockDim.x + 63) >> 6, w = tid >> 6, l = tid & 63;
    const bool own = tid < n;
    uint64_t done0 = 0, done1 = 0;            // pivots taken (the same in every thread)
    auto done = [&](int i) { return (((i < 64) ? (done0 >> i) : (done1 >> (i - 64))) & 1) != 0; };
    auto put = [&](int i, int c, double v) {
        out[i * n + c] = v;
        if (cache) cache[i * n + c] = v;
    };
    double tol = 0.0;
    int c = 0;
    __syncthreads();
    for (; c < n; ++c) {
        // largest remaining diagonal entry; ties go to the smaller index
        double v = (own && !done(tid)) ? (double)M[tid * n + tid] : -1.0;
        int p = tid;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double v2 = __shfl_xor(v, o, 64);
            const int p2 = __shfl_xor(p, o, 64);
            if (v2 > v || (v2 == v && p2 < p)) {
                v = v2;
                p = p2;
            }
        }
        if (l == 0) {
            s_val[c & 1][w] = v;
            s_idx[c & 1][w] = p;
        }
        __syncthreads();
        v = s_val[c & 1][0];
        p = s_idx[c & 1][0];
        for (int u = 1; u < nw; ++u) {
            const double v2 = s_val[c & 1][u];
            const int p2 = s_idx[c & 1][u];
            if (v2 > v || (v2 == v && p2 < p)) {
                v = v2;
                p = p2;
            }
        }
        if (c == 0) tol = (double)n * eps * v;
        if (!(v > tol)) break;                // rank reached (also an all-zero M)
        const double s = 1.0 / sqrt(v);
        if (own) {
            if (done(tid)) {
                put(tid, c, 0.0);
            } else if (tid == p) {
                put(tid, c, v * s);
            } else {
                const double li = (double)M[tid * n + p] * s;
                put(tid, c, li);
                for (int k = 0; k < n; ++k)
                    if (k != p && !done(k)) M[tid * n + k] = (T)((double)M[tid * n + k] - li * ((double)M[p * n + k] * s));
            }
        }
        if (p < 64)
            done0 |= 1ull << p;
        else
            done1 |= 1ull << (p - 64);
        __syncthreads();
    }
    if (own)
        for (int cc = c; cc < n; ++cc) put(tid, cc, 0.0);
}

// The same factorization for n <= NM <= 64 (NM known at compile time): the
// thread of row i keeps that row in registers, the pivot column goes through
// a short LDS vector, and M is only read.
template <int NM, class T>
__device__ __attribute__((noinline)) void rank_reveal_rows(const T *M, int n, double eps, double *out,
                                                           double *cache) {
    static_assert(NM >= 1 && NM <= 64, "one register row of at most 64");
    __shared__ double s_val[16], s_l[NM];
    __shared__ int s_idx[16];
    const int tid = threadIdx.x, nw = (int)(blockDim.x + 63) >> 6, w = tid >> 6, l = tid & 63;
    const bool own = tid < n;
    auto put = [&](int i, int c, double v) {
        out[i * n + c] = v;
        if (cache) cache[i * n + c] = v;
    };
    double r[NM];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NM; ++k) r[k] = (own && k < n) ? (double)M[tid * n + k] : 0.0;
    uint64_t done = 0;                        // pivots taken (the same in every thread)
    double tol = 0.0;
    int c = 0;
    for (; c < n; ++c) {
        const bool live = own && !((done >> tid) & 1);
        double d = 0.0;
#pragma unroll
        for (int k = 0; k < NM; ++k) d = (k == tid) ? r[k] : d;
        double v = live ? d : -1.0;
        int p = tid;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double v2 = __shfl_xor(v, o, 64);
            const int p2 = __shfl_xor(p, o, 64);
            if (v2 > v || (v2 == v && p2 < p)) {
                v = v2;
                p = p2;
            }
        }
        if (l == 0) {
            s_val[w] = v;
            s_idx[w] = p;
        }
        __syncthreads();
        v = s_val[0];
        p = s_idx[0];
        for (int u = 1; u < nw; ++u) {
            const double v2 = s_val[u];
            const int p2 = s_idx[u];
            if (v2 > v || (v2 == v && p2 < p)) {
                v = v2;
                p = p2;
            }
        }
        if (c == 0) tol = (double)n * eps * v;
        if (!(v > tol)) break;                // rank reached (also an all-zero M)
        const double s = 1.0 / sqrt(v);
        double rp = 0.0;
#pragma unroll
        for (int k = 0; k < NM; ++k) rp = (k == p) ? r[k] : rp;
        const double li = (live && tid != p) ? rp * s : 0.0;
        if (own) put(tid, c, !live ? 0.0 : (tid == p ? v * s : li));
        if (tid < NM) s_l[tid] = li;          // 0 for the pivot row and rows already taken
        __syncthreads();
        if (live && tid != p) {
#pragma unroll
            for (int k = 0; k < NM; ++k) r[k] -= li * s_l[k];
        }
        done |= 1ull << p;
    }
    if (own)
        for (int cc = c; cc < n; ++cc) put(tid, cc, 0.0);
}

template <class T>
__device__ __forceinline__ constexpr double unit_roundoff() {
    return sizeof(T) == 4 ? 1.1920928955078125e-07 : 2.220446049250313e-16;
}

// ---------------------------------------------------------------- LDS
// Working set of one workgroup.  RED selects the extra state of Alg. 4.
template <class T, int NX, int NU, bool RED>
struct Smem {
    static constexpr int NW = NX + NU;
    T P[NX * NX];       // cost-to-go Hessian P_{t+1}, overwritten by P_t
    T A[NX * NX];
    T B[NX * NU];
    T W[NX * NW];       // P [A B]; later A'V (RED) or forward-pass staging
    T F[NX * NX];
    T H[NX * NU];       // H_{t+1}, then Y' = (L^{-1} H')' in place
    T G[NU * NU];       // G_{t+1}, then its Cholesky factor L
    T K[RED ? 1 : NU * NX];   // feedback K_{t+1} (solve mode)
    T Psi[NX], av[NX], Pa[NX], pt[NX], gx[NX], x[NX], xn[NX];
    T gw[NU], dinv[NU], kk[NU], wv[NU];
    T V[RED ? NX * NX : 1];   // V_{t+1}
    T Qh[RED ? NX * NX : 1];  // accumulated Q_w_hat
    T BV[RED ? NU * NX : 1];  // B'V, then X = L^{-1} B'V in place
    T v[RED ? NX : 1], Vta[RED ? NX : 1];
    T red[NT / 64];
    T cbar;
    int bad;
};

// Sum of v over the workgroup (all threads must call).
template <class T, class S>
__device__ __forceinline__ T block_sum(T v, S &sm) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sm.red[threadIdx.x >> 6] = v;
    __syncthreads();
    T s = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += sm.red[w];
    return s;
}

// First failure of an instance wins; master-level failures carry stage -1.
__device__ __forceinline__ void record_failure(int32_t *info, int inst, int code, int stage) {
    if (stage < 0) stage = -1;
    if (info) {
        if (atomicCAS(&info[2 * inst], 0, code) == 0) info[2 * inst + 1] = stage;
    }
}

// ================================================================ Alg. 4
// Reduce a subproblem with unknown terminal cost (Alg. 4).  get(s) returns
// local stage s (0..count-1).  Writes the M1 message (A_hat = V_0', B_hat =
// Q_w_hat, a_hat = v_0, Q_x_hat = P_0, l_x_hat = -Psi_0, c_hat = cbar_0) to
// `out`.  The paper's L_{t+1} = -G^{-1} B' V and K_{t+1} enter only through
// products that are formed here from X = L^{-1} B'V and Y = L^{-1} H':
//   L' G L = X' X,   K' B' V = -Y' X,   V' B k = X' z   (z = L^{-1} g_w),
// which are algebraically the lines of Alg. 4.  The constant cbar follows
// the update of Alg. 2 (Alg. 4 uses c_hat = cbar_0 without listing it).
template <class T, int NX, int NU, class Get>
__device__ void reduce_pass(Smem<T, NX, NU, true> &S, Get get, int count, double *out, int32_t *info,
                            int inst, int stage_base, bool rr) {
    constexpr int NW = NX + NU;
    const int tid = threadIdx.x;
    count = uni(count);
    for (int e = tid; e < NX * NX; e += NT) {
        const int i = e / NX, j = e % NX;
        S.P[e] = 0;
        S.V[e] = (i == j) ? T(1) : T(0);
        S.Qh[e] = 0;
    }
    for (int i = tid; i < NX; i += NT) {
        S.Psi[i] = 0;
        S.v[i] = 0;
    }
    if (tid == 0) {
        S.cbar = 0;
        S.bad = 0;
    }
    __syncthreads();
    for (int s = count - 1; s >= 0; --s) {
        const StageSrc src = get(s);
        // -- load A, B, a
        for (int e = tid; e < NX * NX; e += NT) S.A[e] = (T)src.A[e];
        for (int e = tid; e < NX * NU; e += NT) S.B[e] = (T)src.B[e];
        for (int i = tid; i < NX; i += NT) S.av[i] = src.a ? (T)src.a[i] : T(0);
        __syncthreads();
        // -- W = P [A B], P a, Psi - P a, B'V
        mm<NX, NX, NX, false, false>(S.P, NX, S.A, NX, tid, NT,
                                     [&](int i, int j, T acc) { S.W[i * NW + j] = acc; });
        mm<NX, NU, NX, false, false>(S.P, NX, S.B, NU, tid, NT,
                                     [&](int i, int j, T acc) { S.W[i * NW + NX + j] = acc; });
        mm<NU, NX, NX, true, false>(S.B, NU, S.V, NX, tid, NT,
                                    [&](int i, int j, T acc) { S.BV[i * NX + j] = acc; });
        mv<NX, NX, false>(S.P, NX, S.av, tid, NT, [&](int i, T acc) {
            S.Pa[i] = acc;
            S.pt[i] = S.Psi[i] - acc;
        });
        __syncthreads();
        // -- F = Qx + A'PA, H = Qxw + A'PB, G = Qw + B'PB (Alg. 1); g = [A B]'(Psi - Pa)
        mm<NX, NX, NX, true, false>(S.A, NX, S.W, NW, tid, NT,
                                    [&](int i, int j, T acc) { S.F[i * NX + j] = (T)src.Qx[i * NX + j] + acc; });
        mm<NX, NU, NX, true, false>(S.A, NX, S.W + NX, NW, tid, NT, [&](int i, int j, T acc) {
            S.H[i * NU + j] = (src.Qxw ? (T)src.Qxw[i * NU + j] : T(0)) + acc;
        });
        mm<NU, NU, NX, true, false>(S.B, NU, S.W + NX, NW, tid, NT,
                                    [&](int i, int j, T acc) { S.G[i * NU + j] = (T)src.Qw[i * NU + j] + acc; });
        mv<NX, NX, true>(S.A, NX, S.pt, tid, NT,
                         [&](int i, T acc) { S.gx[i] = acc - (src.lx ? (T)src.lx[i] : T(0)); });
        mv<NU, NX, true>(S.B, NU, S.pt, tid, NT,
                         [&](int i, T acc) { S.gw[i] = acc - (src.lw ? (T)src.lw[i] : T(0)); });
        mv<NX, NX, true>(S.V, NX, S.av, tid, NT, [&](int i, T acc) { S.Vta[i] = acc; });
        {
            // cbar += 1/2 a'Pa - Psi'a + c   (Alg. 2, with P_{t+1}, Psi_{t+1})
            T part = 0;
            for (int i = tid; i < NX; i += NT) part += T(0.5) * S.av[i] * S.Pa[i] - S.Psi[i] * S.av[i];
            const T tot = block_sum(part, S);
            if (tid == 0) S.cbar += tot + (T)src.c;
        }
        __syncthreads();
        // -- factor G (wave 0) while the other waves form A'V into W
        if (tid < 64) {
            const int f = chol_wave<NU>(S.G, S.dinv);
            if (f && tid == 0) S.bad = 1;
        } else {
            mm<NX, NX, NX, true, false>(S.A, NX, S.V, NX, tid - 64, NT - 64,
                                        [&](int i, int j, T acc) { S.W[i * NX + j] = acc; });
        }
        __syncthreads();
        if (S.bad && tid == 0) {
            record_failure(info, inst, stage_base < 0 ? 3 : 2, stage_base < 0 ? -1 : stage_base + s);
            S.bad = 0;
        }
        // -- column solves: Y' rows (L^{-1}H'), X columns (L^{-1}B'V), z = L^{-1} g_w
        if (tid < NX) {
            T y[NU];
#pragma unroll
            for (int r = 0; r < NU; ++r) y[r] = S.H[tid * NU + r];
            trsv_l<NU>(S.G, S.dinv, y);
#pragma unroll
            for (int r = 0; r < NU; ++r) S.H[tid * NU + r] = y[r];
        } else if (tid < 2 * NX) {
            const int c = tid - NX;
            T y[NU];
#pragma unroll
            for (int r = 0; r < NU; ++r) y[r] = S.BV[r * NX + c];
            trsv_l<NU>(S.G, S.dinv, y);
#pragma unroll
            for (int r = 0; r < NU; ++r) S.BV[r * NX + c] = y[r];
        } else if (tid == 2 * NX) {
            T y[NU];
#pragma unroll
            for (int r = 0; r < NU; ++r) y[r] = S.gw[r];
            trsv_l<NU>(S.G, S.dinv, y);
#pragma unroll
            for (int r = 0; r < NU; ++r) S.gw[r] = y[r];
        }
        __syncthreads();
        // -- P = F - Y'Y (symmetrised), Q_w_hat += X'X, V = A'V - Y'X,
        //    Psi = g_x - Y'z, v += V'a + X'z, cbar -= 1/2 z'z
        mm<NX, NX, NU, false, true>(S.H, NU, S.H, NU, tid, NT, [&](int i, int j, T acc) {
            S.P[i * NX + j] = T(0.5) * (S.F[i * NX + j] + S.F[j * NX + i]) - acc;
        });
        mm<NX, NX, NU, true, false>(S.BV, NX, S.BV, NX, tid, NT,
                                    [&](int i, int j, T acc) { S.Qh[i * NX + j] += acc; });
        mm<NX, NX, NU, false, false>(S.H, NU, S.BV, NX, tid, NT,
                                     [&](int i, int j, T acc) { S.V[i * NX + j] = S.W[i * NX + j] - acc; });
        mv<NX, NU, false>(S.H, NU, S.gw, tid, NT, [&](int i, T acc) { S.Psi[i] = S.gx[i] - acc; });
        mv<NX, NU, true>(S.BV, NX, S.gw, tid, NT, [&](int i, T acc) { S.v[i] += S.Vta[i] + acc; });
        {
            T part = 0;
            for (int r = tid; r < NU; r += NT) part += S.gw[r] * S.gw[r];
            const T tot = block_sum(part, S);
            if (tid == 0) S.cbar -= T(0.5) * tot;
        }
        __syncthreads();
    }
    // -- M1 message to the parent (Alg. 4 last lines, Alg. 5 "send")
    const SlotLayout L{NX};
    for (int e = tid; e < NX * NX; e += NT) {
        const int i = e / NX, j = e % NX;
        out[L.A() + e] = (double)S.V[j * NX + i];     // A_hat = V_0'
        if (!rr) out[L.Qw() + e] = (double)S.Qh[e];
        out[L.Qx() + e] = (double)S.P[e];
    }
    for (int i = tid; i < NX; i += NT) {
        out[L.a() + i] = (double)S.v[i];
        out[L.lx() + i] = -(double)S.Psi[i];
    }
    if (tid == 0) out[L.c()] = (double)S.cbar;
    if (rr) rank_reveal_rows<NX>(S.Qh, NX, unit_roundoff<T>(), out + L.Qw(), nullptr);
}

// ========================================================= Alg. 1-2 (-3)
// Backward Riccati pass over `count` stages from a known terminal cost
// (P_N, Psi_N, cbar_N already in S.P, S.Psi, S.cbar).  With SOLVE the
// feedback K_{t+1}, k_{t+1} is formed and handed to `store(s, S)` together
// with P_t, Psi_t after each stage, and `pre(s, S)` sees P_{t+1}, Psi_{t+1},
// cbar_{t+1} before each stage.  Without SOLVE it is the elimination of the
// last subproblem (Sec. 4.2) and leaves P_0, Psi_0, cbar_0 in LDS.
template <bool SOLVE, class T, int NX, int NU, class Get, class Pre, class Store>
__device__ void backward_pass(Smem<T, NX, NU, false> &S, Get get, int count, int32_t *info, int inst,
                              int stage_base, int fail_code, Pre pre, Store store) {
    constexpr int NW = NX + NU;
    const int tid = threadIdx.x;
    count = uni(count);
    if (tid == 0) S.bad = 0;
    __syncthreads();
    for (int s = count - 1; s >= 0; --s) {
        const StageSrc src = get(s);
        pre(s, S);
        for (int e = tid; e < NX * NX; e += NT) S.A[e] = (T)src.A[e];
        for (int e = tid; e < NX * NU; e += NT) S.B[e] = (T)src.B[e];
        for (int i = tid; i < NX; i += NT) S.av[i] = src.a ? (T)src.a[i] : T(0);
        __syncthreads();
        mm<NX, NX, NX, false, false>(S.P, NX, S.A, NX, tid, NT,
                                     [&](int i, int j, T acc) { S.W[i * NW + j] = acc; });
        mm<NX, NU, NX, false, false>(S.P, NX, S.B, NU, tid, NT,
                                     [&](int i, int j, T acc) { S.W[i * NW + NX + j] = acc; });
        mv<NX, NX, false>(S.P, NX, S.av, tid, NT, [&](int i, T acc) {
            S.Pa[i] = acc;
            S.pt[i] = S.Psi[i] - acc;
        });
        __syncthreads();
        mm<NX, NX, NX, true, false>(S.A, NX, S.W, NW, tid, NT,
                                    [&](int i, int j, T acc) { S.F[i * NX + j] = (T)src.Qx[i * NX + j] + acc; });
        mm<NX, NU, NX, true, false>(S.A, NX, S.W + NX, NW, tid, NT, [&](int i, int j, T acc) {
            S.H[i * NU + j] = (src.Qxw ? (T)src.Qxw[i * NU + j] : T(0)) + acc;
        });
        mm<NU, NU, NX, true, false>(S.B, NU, S.W + NX, NW, tid, NT,
                                    [&](int i, int j, T acc) { S.G[i * NU + j] = (T)src.Qw[i * NU + j] + acc; });
        mv<NX, NX, true>(S.A, NX, S.pt, tid, NT,
                         [&](int i, T acc) { S.gx[i] = acc - (src.lx ? (T)src.lx[i] : T(0)); });
        mv<NU, NX, true>(S.B, NU, S.pt, tid, NT,
                         [&](int i, T acc) { S.gw[i] = acc - (src.lw ? (T)src.lw[i] : T(0)); });
        {
            T part = 0;
            for (int i = tid; i < NX; i += NT) part += T(0.5) * S.av[i] * S.Pa[i] - S.Psi[i] * S.av[i];
            const T tot = block_sum(part, S);
            if (tid == 0) S.cbar += tot + (T)src.c;
        }
        __syncthreads();
        if (tid < 64) {
            const int f = chol_wave<NU>(S.G, S.dinv);
            if (f && tid == 0) S.bad = 1;
        }
        __syncthreads();
        if (S.bad && tid == 0) {
            record_failure(info, inst, fail_code, stage_base < 0 ? -1 : stage_base + s);
            S.bad = 0;
        }
        if (tid < NX) {
            T y[NU];
#pragma unroll
            for (int r = 0; r < NU; ++r) y[r] = S.H[tid * NU + r];
            trsv_l<NU>(S.G, S.dinv, y);
#pragma unroll
            for (int r = 0; r < NU; ++r) S.H[tid * NU + r] = y[r];
            if constexpr (SOLVE) {
                // K_{t+1} = -G^{-1} H' : column tid of K = -L^{-T} y
                trsv_lt<NU>(S.G, S.dinv, y);
#pragma unroll
                for (int r = 0; r < NU; ++r) S.K[r * NX + tid] = -y[r];
            }
        } else if (tid == NX) {
            T y[NU];
#pragma unroll
            for (int r = 0; r < NU; ++r) y[r] = S.gw[r];
            trsv_l<NU>(S.G, S.dinv, y);
#pragma unroll
            for (int r = 0; r < NU; ++r) S.gw[r] = y[r];
            if constexpr (SOLVE) {
                trsv_lt<NU>(S.G, S.dinv, y);   // k_{t+1} = G^{-1}(B'Psi - l_w - B'Pa)
#pragma unroll
                for (int r = 0; r < NU; ++r) S.kk[r] = y[r];
            }
        }
        __syncthreads();
        mm<NX, NX, NU, false, true>(S.H, NU, S.H, NU, tid, NT, [&](int i, int j, T acc) {
            S.P[i * NX + j] = T(0.5) * (S.F[i * NX + j] + S.F[j * NX + i]) - acc;
        });
        mv<NX, NU, false>(S.H, NU, S.gw, tid, NT, [&](int i, T acc) { S.Psi[i] = S.gx[i] - acc; });
        {
            T part = 0;
            for (int r = tid; r < NU; r += NT) part += S.gw[r] * S.gw[r];
            const T tot = block_sum(part, S);
            if (tid == 0) S.cbar -= T(0.5) * tot;
        }
        __syncthreads();
        store(s, S);
        // every loop that contains barriers ends on a barrier, so that its
        // back edge is taken by all lanes together
        __syncthreads();
    }
}

// Forward recursion (Alg. 3) over `count` stages from x in S.x; `fetch(s, S)`
// loads K_{t+1} into S.K, k_{t+1} into S.kk (and whatever `emit` needs),
// emit(s, S) writes the per-stage outputs after w and x_{t+1} are formed
// (S.x = x_t, S.wv = w_t, S.xn = x_{t+1}).
template <class T, int NX, int NU, class Get, class Fetch, class Emit>
__device__ void forward_pass(Smem<T, NX, NU, false> &S, Get get, int count, Fetch fetch, Emit emit) {
    const int tid = threadIdx.x;
    count = uni(count);
    for (int s = 0; s < count; ++s) {
        const StageSrc src = get(s);
        fetch(s, S);
        for (int e = tid; e < NX * NX; e += NT) S.A[e] = (T)src.A[e];
        for (int e = tid; e < NX * NU; e += NT) S.B[e] = (T)src.B[e];
        for (int i = tid; i < NX; i += NT) S.av[i] = src.a ? (T)src.a[i] : T(0);
        __syncthreads();
        mv<NU, NX, false>(S.K, NX, S.x, tid, NT, [&](int r, T acc) { S.wv[r] = S.kk[r] + acc; });
        __syncthreads();
        for (int i = tid; i < NX; i += NT) {
            T acc = S.av[i];
#pragma unroll 4
            for (int k = 0; k < NX; ++k) acc += S.A[i * NX + k] * S.x[k];
#pragma unroll 4
            for (int r = 0; r < NU; ++r) acc += S.B[i * NU + r] * S.wv[r];
            S.xn[i] = acc;
        }
        __syncthreads();
        emit(s, S);
        __syncthreads();
        for (int i = tid; i < NX; i += NT) S.x[i] = S.xn[i];
        __syncthreads();
    }
}

}  // namespace rs
