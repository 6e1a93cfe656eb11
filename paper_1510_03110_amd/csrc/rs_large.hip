// Large-block kernels of the parallel Riccati solve: any n_x, n_u up to 128
// without a register- and LDS-resident specialisation (the n_x = 64 and
// n_x = 128 problems; also the stored factorization of the small shapes
// whose fused solve has no matrix-core form).  A 64 x 64 FP64 stage already needs
// about 260 KB of working set, more than a CU's LDS, so here the matrices of a
// work unit live in a per-workgroup workspace in global memory (L2-resident
// while the unit runs) and only vectors use LDS.  Sizes are run-time values.
//
// The family implements the factor / solve split; the fused FP64 solve of
// these shapes is the stored factorization followed by the solve on it.
//   kl_leaf_up     one workgroup per leaf (grid-stride): matrix lines of
//                  Alg. 4 or of the last-leaf elimination; up records and the
//                  matrix part of the M1 message
//   kl_tree        work-queue kernel over the master levels: Alg. 4 on master
//                  groups (Alg. 5), elimination of the last group, and the
//                  factorization of the top subproblem (Alg. 6; below the
//                  top the down pass is kw_tree's superposition sweep on the
//                  up records, or, with RS_PLAN_REFACTOR_DOWN, a second
//                  factorization from the parent's message)
//   kl_leaf_down   whole-problem leaves: Alg. 1 with the true terminal
//   kw_leaf_up / kw_tree / kw_leaf_down
//                  the vector lines of the same passes and the forward
//                  recursion (Alg. 2-3, vector part of Alg. 4), one
//                  workgroup per unit
//   kw_residual / kw_update
//                  FP64 KKT residual and update of iterative refinement
//
// Every dense product of a stage is a list of 16x16 output tiles on the
// matrix cores (v_mfma_f64_16x16x4f64, or the f32 form for FP32 factors),
// tile t of a product going to wave t mod 8; at n_x > 64 the operands come
// through LDS panels shared by the workgroup (gemm_panel), at n_x <= 64 each
// tile reads its own strips (gemm_tile).  Products of one phase are
// independent, and a workgroup barrier separates phases.  Per stage:
//   W = P [A B];  (Alg. 4) B'V, A'V
//   F = Qx + A'W_A,  H = Qxw + A'W_B,  G = Qw + B'W_B                 (Alg. 1)
//   G = L L', L^{-1}  (blocked: 16 x 16 diagonal factorizations by one
//                      wavefront, panels and trailing updates on MFMA)
//   Y' = H L^{-T};  (Alg. 4) X = L^{-1} B'V
//   P = F - Y'Y,  K = -L^{-T} Y;  (Alg. 4) Q_w_hat += X'X, V = A'V - Y'X,
//   L_t = -L^{-T} X
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rs_launch.hpp"
#include "rs_mfma.hpp"
#include "rs_vec.hpp"

namespace rs {
namespace lb {

using mf::lane;
using mf::MT;
using mf::v4_t;
using mf::wave;

constexpr int SPIN_LIMIT = 1 << 26;

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

// ------------------------------------------------------------- workspace
// Matrices of one work unit, row-major, elements of T:
//   P V Qh F AV (n x n) | AB W (n x (n+m)) | H HY (n x m) | BV X (m x n) |
//   G Li LiT Lp (m x m) | D DT (16 x 16) | Tm (m x 16)
template <class T>
struct WS {
    int n, m, nw;
    T *P, *V, *Qh, *F, *AV, *AB, *W, *H, *HY, *BV, *X, *G, *Li, *LiT, *Lp, *D, *DT, *Tm;
    __device__ void bind(T *b, int n_, int m_) {
        n = n_;
        m = m_;
        nw = n + m;
        const int64_t nn = (int64_t)n * n, nm = (int64_t)n * m, mm = (int64_t)m * m, nwn = (int64_t)n * nw;
        P = b;
        V = P + nn;
        Qh = V + nn;
        F = Qh + nn;
        AV = F + nn;
        AB = AV + nn;
        W = AB + nwn;
        H = W + nwn;
        HY = H + nm;
        BV = HY + nm;
        X = BV + nm;
        G = X + nm;
        Li = G + mm;
        LiT = Li + mm;
        Lp = LiT + mm;
        D = Lp + mm;
        DT = D + 256;
        Tm = DT + 256;
    }
};

}  // namespace lb

size_t large_unit_bytes(int nx, int nu) {
    // the master levels factor n x n blocks (m = n), so a unit holds the
    // larger of the two working sets
    auto elems = [](int64_t n, int64_t m) {
        return 5 * n * n + 2 * n * (n + m) + 4 * n * m + 4 * m * m + 512 + 16 * m;
    };
    const int64_t e = std::max(elems(nx, nu), elems(nx, nx));
    return (size_t)(((e * 8) + 255) & ~(int64_t)255);
}

namespace lb {

// Threads and wavefronts of the workgroup: the matrix kernels run LB_MT
// threads (8 wavefronts), so twice as many 16x16 tiles of a product are in
// flight per work unit as with 4.
constexpr int LB_MT = 512;
__device__ __forceinline__ int nthr() { return (int)blockDim.x; }
__device__ __forceinline__ int nwav() { return (int)(blockDim.x >> 6); }

// Orders one wavefront's global-memory traffic (stores of some lanes before
// loads of others).
__device__ __forceinline__ void wave_gfence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Where the result of a large-block product goes: element (i, j) of
// v = sgn * opA(A) opB(B) + D is stored to C and, when given, to the record R;
// with `sym` (the lower products of symmetric results, i >= j) also to (j, i).
// D is problem data (FP64) or a workspace matrix (element type T), or none.
template <class T>
struct Ep {
    T *C = nullptr;
    int ldc = 0;
    const double *D64 = nullptr;
    const T *DT = nullptr;
    int ldd = 0;
    T sgn = T(1);
    bool sym = false;
    T *R = nullptr;
    int ldr = 0;
};

// Global-memory views of the operands of an out-of-line product (its pointer
// arguments would otherwise be generic, and generic loads are also counted
// with the LDS accesses).
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gview(const T *p) {
    return (const __attribute__((address_space(1))) T *)p;
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gview(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}

template <class T>
__device__ __forceinline__ void put(const Ep<T> &e, int i, int j, T c) {
    T v = e.sgn * c;
    if (e.D64)
        v += (T)gview(e.D64)[(int64_t)i * e.ldd + j];
    else if (e.DT)
        v += gview(e.DT)[(int64_t)i * e.ldd + j];
    if (e.C) {
        gview(e.C)[(int64_t)i * e.ldc + j] = v;
        if (e.sym) gview(e.C)[(int64_t)j * e.ldc + i] = v;
    }
    if (e.R) {
        gview(e.R)[(int64_t)i * e.ldr + j] = v;
        if (e.sym && i != j) gview(e.R)[(int64_t)j * e.ldr + i] = v;
    }
}

// Operand panels of the large-block products, staged in LDS: a 16-wide
// inner panel of A (up to 128 rows, row pitch 17) and of B (16 rows of up to
// 128 columns, pitch 144), shared by every wavefront of the workgroup.  The
// pitches keep the MFMA operand reads nearly free of bank conflicts: rows of
// the A panel 17 doubles apart fall on distinct banks for the 16 lanes of a
// row group, and the two row groups of a half-wave read B rows 32 banks apart.
constexpr int GP_K = 16, GP_M = 128, GP_N = 128, GP_AP = GP_K + 1, GP_BP = GP_N + 16;
constexpr int GP_ELEMS = GP_M * GP_AP + GP_K * GP_BP;
// products with fewer 16 x 16 tiles than this take the per-tile form
constexpr int GP_MIN_TILES = 32;
__shared__ double gp_sm[GP_ELEMS];

// C = opA(A) opB(B): M x N (M <= 128, any N; with `lower` square and
// N <= 128), inner size K; the result goes through the epilogue `ep`.
// opA(i,k) = TA ? A[k*lda+i] : A[i*lda+k], opB(k,j) = TB ? B[j*ldb+k] :
// B[k*ldb+j].  The result is formed in column chunks of up to 128; for each
// chunk the workgroup walks the inner dimension in panels of 16: its threads
// load the A and B panels (zero-padded to whole 16 x 16 tiles, loads laid out
// along the operand's contiguous direction) into LDS, and each wavefront
// accumulates its 16 x 16 tiles (tile t goes to wave t mod 8, at most 8 per
// wave) from there while the next panel's loads are in flight: one memory
// round trip per panel of 16 for every tile of the chunk at once, where a
// tile that read its own operand strips needed one per 32 of inner size.
// With `lower` only the tiles on and below the diagonal are formed and only
// the elements with i >= j are put.  Small products (fewer than
// GP_MIN_TILES tiles, such as G at n_u <= 64) skip the panels, and each wave
// reads its tiles' operand strips itself.  One out-of-line body per operand
// layout keeps the stage's code within the instruction cache.  Every thread
// of the workgroup must call it (it synchronizes the workgroup).
template <bool TA, bool TB, class T>
__device__ __attribute__((noinline)) void gemm_panel(int M, int N, int K, const T *A, int lda, const T *B, int ldb,
                                                     bool lower, Ep<T> ep) {
    static_assert(LB_MT == 512, "eight wavefronts: at most eight 16 x 16 tiles of a chunk per wave");
    constexpr int QMAX = (GP_M / 16) * (GP_N / 16) / (LB_MT / 64);
    constexpr int EA = GP_M * GP_K / LB_MT, EB = GP_K * GP_N / LB_MT;
    const auto gA = gview(A);
    const auto gB = gview(B);
    T *As = reinterpret_cast<T *>(gp_sm), *Bs = As + GP_M * GP_AP;
    const int tid = threadIdx.x, w = wave(), l = lane(), r16 = l & 15, k4 = l >> 4;
    const int tm = (M + 15) >> 4, Mp = 16 * tm;
    if ((lower ? tm * (tm + 1) / 2 : tm * ((N + 15) >> 4)) < GP_MIN_TILES) {
        // small product: each wave forms its tiles from operand strips read
        // straight from memory (no barriers; the panels would cost more in
        // synchronization than they save)
        const int tn = (N + 15) >> 4, nt = lower ? tm * (tm + 1) / 2 : tm * tn;
        for (int t = w; t < nt; t += LB_MT / 64) {
            int ti, tj;
            if (lower) {
                mf::lower_tile(t, ti, tj);
            } else {
                ti = t / tn;
                tj = t - ti * tn;
            }
            const int i = 16 * ti + r16, j = 16 * tj + r16;
            const bool iv = i < M, jv = j < N;
            v4_t<T> acc = mf::zero4<T>();
#pragma unroll 2
            for (int k0 = 0; k0 < K; k0 += 16) {
                T a[4], b[4];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int k = k0 + 4 * s + k4;
                    a[s] = (iv && k < K) ? (TA ? gA[(int64_t)k * lda + i] : gA[(int64_t)i * lda + k]) : T(0);
                    b[s] = (jv && k < K) ? (TB ? gB[(int64_t)j * ldb + k] : gB[(int64_t)k * ldb + j]) : T(0);
                }
#pragma unroll
                for (int s = 0; s < 4; ++s) acc = MT<T>::mfma(a[s], b[s], acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ii = mf::trow<T>(ti, r), jj = mf::tcol(tj);
                if (ii < M && jj < N && (!lower || ii >= jj)) put(ep, ii, jj, acc[r]);
            }
        }
        return;
    }
    for (int n0 = 0; n0 < N; n0 += GP_N) {
        const int NC = N - n0 < GP_N ? N - n0 : GP_N, tn = (NC + 15) >> 4, Np = 16 * tn;
        const int nt = lower ? tm * (tm + 1) / 2 : tm * tn;
        int ti[QMAX], tj[QMAX];
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
            const int t = w + 8 * q;
            if (lower) {
                mf::lower_tile(t < nt ? t : 0, ti[q], tj[q]);
            } else {
                ti[q] = t / tn;
                tj[q] = t - ti[q] * tn;
            }
        }
        v4_t<T> acc[QMAX];
#pragma unroll
        for (int q = 0; q < QMAX; ++q) acc[q] = mf::zero4<T>();
        // panel element e of A: (row, inner index) along A's contiguous
        // direction; of B: (inner index, column) along B's
        auto a_at = [&](int e, int &m, int &kk) {
            if (TA) {
                kk = e / Mp;
                m = e - kk * Mp;
            } else {
                m = e >> 4;
                kk = e & 15;
            }
        };
        auto b_at = [&](int e, int &kk, int &n) {
            if (TB) {
                n = e >> 4;
                kk = e & 15;
            } else {
                kk = e / Np;
                n = e - kk * Np;
            }
        };
        T ra[EA], rb[EB];
        auto fetch = [&](int k0) {
#pragma unroll
            for (int u = 0; u < EA; ++u) {
                const int e = tid + u * LB_MT;
                int m, kk;
                a_at(e, m, kk);
                const int k = k0 + kk;
                ra[u] = (e < Mp * GP_K && m < M && k < K) ? (TA ? gA[(int64_t)k * lda + m] : gA[(int64_t)m * lda + k])
                                                          : T(0);
            }
#pragma unroll
            for (int u = 0; u < EB; ++u) {
                const int e = tid + u * LB_MT;
                int kk, n;
                b_at(e, kk, n);
                const int k = k0 + kk, j = n0 + n;
                rb[u] = (e < Np * GP_K && n < NC && k < K) ? (TB ? gB[(int64_t)j * ldb + k] : gB[(int64_t)k * ldb + j])
                                                           : T(0);
            }
        };
        fetch(0);
        for (int k0 = 0; k0 < K; k0 += GP_K) {
            __syncthreads();      // every wave is done with the previous panel
#pragma unroll
            for (int u = 0; u < EA; ++u) {
                const int e = tid + u * LB_MT;
                int m, kk;
                a_at(e, m, kk);
                if (e < Mp * GP_K) As[m * GP_AP + kk] = ra[u];
            }
#pragma unroll
            for (int u = 0; u < EB; ++u) {
                const int e = tid + u * LB_MT;
                int kk, n;
                b_at(e, kk, n);
                if (e < Np * GP_K) Bs[kk * GP_BP + n] = rb[u];
            }
            __syncthreads();
            if (k0 + GP_K < K) fetch(k0 + GP_K);
#pragma unroll
            for (int q = 0; q < QMAX; ++q) {
                if (w + 8 * q < nt) {
                    const T *ap = As + (16 * ti[q] + r16) * GP_AP + k4;
                    const T *bp = Bs + k4 * GP_BP + 16 * tj[q] + r16;
#pragma unroll
                    for (int s = 0; s < 4; ++s) acc[q] = MT<T>::mfma(ap[4 * s], bp[4 * s * GP_BP], acc[q]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
            if (w + 8 * q < nt) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = mf::trow<T>(ti[q], r), j = n0 + mf::tcol(tj[q]);
                    if (i < M && j < N && (!lower || i >= j)) put(ep, i, j, acc[q][r]);
                }
            }
        }
    }
    __syncthreads();      // the results are visible to the workgroup
}

// Stages with n_x <= 64 (products of at most 24 tiles), inline with the
// epilogue as a functor:
// C = opA(A) opB(B): M x N, inner size K (any sizes; edge tiles are padded
// with zeros on load).  opA(i,k) = TA ? A[k*lda+i] : A[i*lda+k], opB(k,j) =
// TB ? B[j*ldb+k] : B[k*ldb+j].  16x16 tile t goes to wave t mod 8; every
// element (i, j) of the result with i < M, j < N is handed to epi(i, j, c).
// With `lower` (square results) only the tiles on and below the diagonal are
// formed, and epi must use the elements with i >= j.
template <bool TA, bool TB, class T, class Epi>
__device__ __forceinline__ void gemm_tile(int M, int N, int K, const T *__restrict__ A, int lda, const T *__restrict__ B,
                                     int ldb, bool lower, Epi epi) {
    const int tm = (M + 15) >> 4, tn = (N + 15) >> 4;
    const int nt = lower ? tm * (tm + 1) / 2 : tm * tn;
    const int l = lane(), r16 = l & 15, k4 = l >> 4;
    for (int t = wave(); t < nt; t += nwav()) {
        int ti, tj;
        if (lower) {
            mf::lower_tile(t, ti, tj);
        } else {
            ti = t / tn;
            tj = t - ti * tn;
        }
        const int i = 16 * ti + r16, j = 16 * tj + r16;
        const bool iv = i < M, jv = j < N;
        v4_t<T> acc = mf::zero4<T>();
#pragma unroll 2
        for (int k0 = 0; k0 < K; k0 += 16) {
            T a[4], b[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = k0 + 4 * s + k4;
                a[s] = (iv && k < K) ? (TA ? A[(int64_t)k * lda + i] : A[(int64_t)i * lda + k]) : T(0);
                b[s] = (jv && k < K) ? (TB ? B[(int64_t)j * ldb + k] : B[(int64_t)k * ldb + j]) : T(0);
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) acc = MT<T>::mfma(a[s], b[s], acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ii = mf::trow<T>(ti, r), jj = mf::tcol(tj);
            if (ii < M && jj < N) epi(ii, jj, acc[r]);
        }
    }
}

// BF16 operands (round to nearest even of the FP32 value; finite inputs).
__device__ __forceinline__ short to_bf16(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// gemm with operands rounded to BF16 and FP32 accumulation
// (v_mfma_f32_16x16x16_bf16: lane l holds A(l % 16, 4 (l / 16) + q) and
// B(4 (l / 16) + q, l % 16), q = 0..3; the result layout is the FP32 one).
template <bool TA, bool TB, class Epi>
__device__ __forceinline__ void gemm_bf16(int M, int N, int K, const float *__restrict__ A, int lda,
                                          const float *__restrict__ B, int ldb, bool lower, Epi epi) {
    typedef short s4 __attribute__((ext_vector_type(4)));
    const int tm = (M + 15) >> 4, tn = (N + 15) >> 4;
    const int nt = lower ? tm * (tm + 1) / 2 : tm * tn;
    const int l = lane(), r16 = l & 15, k4 = l >> 4;
    for (int t = wave(); t < nt; t += nwav()) {
        int ti, tj;
        if (lower) {
            mf::lower_tile(t, ti, tj);
        } else {
            ti = t / tn;
            tj = t - ti * tn;
        }
        const int i = 16 * ti + r16, j = 16 * tj + r16;
        const bool iv = i < M, jv = j < N;
        v4_t<float> acc = mf::zero4<float>();
        for (int k0 = 0; k0 < K; k0 += 16) {
            s4 a, b;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = k0 + 4 * k4 + q;
                const float av = (iv && k < K) ? (TA ? A[(int64_t)k * lda + i] : A[(int64_t)i * lda + k]) : 0.0f;
                const float bv = (jv && k < K) ? (TB ? B[(int64_t)j * ldb + k] : B[(int64_t)k * ldb + j]) : 0.0f;
                a[q] = to_bf16(av);
                b[q] = to_bf16(bv);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ii = mf::trow<float>(ti, r), jj = mf::tcol(tj);
            if (ii < M && jj < N) epi(ii, jj, acc[r]);
        }
    }
}

// The products of the stage that may run on BF16 operands.
template <bool BF, bool TA, bool TB, class T, class Epi>
__device__ __forceinline__ void gemm_big(int M, int N, int K, const T *A, int lda, const T *B, int ldb, bool lower,
                                         Epi epi) {
    if constexpr (BF)
        gemm_bf16<TA, TB>(M, N, K, A, lda, B, ldb, lower, epi);
    else
        gemm_tile<TA, TB>(M, N, K, A, lda, B, ldb, lower, epi);
}
template <bool BF, bool TA, bool TB, class T>
__device__ __forceinline__ void gemm_big_panel(int M, int N, int K, const T *A, int lda, const T *B, int ldb,
                                               bool lower, const Ep<T> &ep) {
    if constexpr (BF)
        gemm_bf16<TA, TB>(M, N, K, A, lda, B, ldb, lower, [&](int i, int j, float c) {
            if (!lower || i >= j) put(ep, i, j, c);
        });
    else
        gemm_panel<TA, TB>(M, N, K, A, lda, B, ldb, lower, ep);
}

// Epilogue descriptors: store to C (leading dimension ldc); plus a
// symmetric addend, a sign or a record copy.
template <class T>
__device__ __forceinline__ Ep<T> to(T *C, int ldc) {
    Ep<T> e;
    e.C = C;
    e.ldc = ldc;
    return e;
}

// acc += opA(A) opB(B) for one 16 x 16 x 16 block with only the first ri
// rows, rk inner indices and rj columns taken (the rest read as zero).
// opA(i,k) = A[i*lda+k]; opB(k,j) = TB ? B[j*ldb+k] : B[k*ldb+j].
template <bool TB, class T>
__device__ __forceinline__ v4_t<T> blk16(v4_t<T> acc, const T *A, int lda, const T *B, int ldb, int ri, int rk,
                                         int rj) {
    const int l = lane(), r16 = l & 15, k4 = l >> 4;
    T a[4], b[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k = 4 * s + k4;
        a[s] = (r16 < ri && k < rk) ? A[(int64_t)r16 * lda + k] : T(0);
        b[s] = (r16 < rj && k < rk) ? (TB ? B[(int64_t)r16 * ldb + k] : B[(int64_t)k * ldb + r16]) : T(0);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) acc = MT<T>::mfma(a[s], b[s], acc);
    return acc;
}

// Blocked Cholesky factorization G = L L' ("a factorization of G", Alg. 1)
// and the explicit inverse (any m <= 128).  Right-looking over 16-wide block
// columns: the diagonal block (padded with the identity past m) is factored
// and inverted by one wavefront (chol_inv_wave), the panel below it is
// L_ik = G_ik L_kk^{-T}, and the trailing lower blocks are updated
// G_ij -= L_ik L_jk'.  The inverse follows block row by block row:
// X_ii = L_ii^{-1}, X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj.  On return
// Li = L^{-1} and LiT = L^{-T} (row-major, zeros above / below the
// diagonal); G is overwritten.  *bad is set if a pivot failed.  Every thread
// must call it; it ends with a workgroup barrier.
template <class T>
__device__ void chol_inv(WS<T> &S, int m, int *bad) {
    const int nb = (m + 15) >> 4, tid = threadIdx.x, w = wave(), l = lane();
    T *G = S.G, *Li = S.Li, *Lp = S.Lp, *D = S.D, *DT = S.DT;
    auto rows = [&](int b) { return m - 16 * b < 16 ? m - 16 * b : 16; };
    for (int kb = 0; kb < nb; ++kb) {
        const int rk = rows(kb);
        if (w == 0) {
            for (int e = l; e < 256; e += 64) {
                const int i = e / 16, j = e % 16;
                D[e] = (i < rk && j < rk) ? G[(int64_t)(16 * kb + i) * m + 16 * kb + j] : (i == j ? T(1) : T(0));
            }
            wave_gfence();
            const int f = mf::chol_inv_wave<16>(D, DT);      // D <- L_kk^{-1}, DT <- L_kk^{-T}
            if (f && l == 0) *bad = 1;
        }
        __syncthreads();
        // panel below the diagonal block, then the trailing lower blocks
        const int np = nb - kb - 1;
        for (int t = w; t < np; t += nwav()) {
            const int ib = kb + 1 + t, ri = rows(ib);
            const v4_t<T> acc = blk16<false>(mf::zero4<T>(), G + (int64_t)16 * ib * m + 16 * kb, m, DT, 16, ri, rk, rk);
            mf::tile_for<T>(0, 0, [&](int r, int i, int j) {
                if (i < ri && j < rk) Lp[(int64_t)(16 * ib + i) * m + 16 * kb + j] = acc[r];
            });
        }
        for (int e = tid; e < 256; e += nthr()) {
            const int i = e / 16, j = e % 16;
            if (i < rk && j < rk) Li[(int64_t)(16 * kb + i) * m + 16 * kb + j] = D[e];
        }
        __syncthreads();
        const int nt = np * (np + 1) / 2;
        for (int t = w; t < nt; t += nwav()) {
            int a, b;
            mf::lower_tile(t, a, b);
            const int ib = kb + 1 + a, jb = kb + 1 + b, ri = rows(ib), rj = rows(jb);
            const v4_t<T> acc = blk16<true>(mf::zero4<T>(), Lp + (int64_t)16 * ib * m + 16 * kb, m,
                                            Lp + (int64_t)16 * jb * m + 16 * kb, m, ri, rk, rj);
            mf::tile_for<T>(0, 0, [&](int r, int i, int j) {
                if (i < ri && j < rj) G[(int64_t)(16 * ib + i) * m + 16 * jb + j] -= acc[r];
            });
        }
        __syncthreads();
    }
    // block rows of the inverse
    for (int ib = 1; ib < nb; ++ib) {
        const int ri = rows(ib);
        for (int jb = w; jb < ib; jb += nwav()) {
            v4_t<T> acc = mf::zero4<T>();
            for (int kb = jb; kb < ib; ++kb)
                acc = blk16<false>(acc, Lp + (int64_t)16 * ib * m + 16 * kb, m, Li + (int64_t)16 * kb * m + 16 * jb, m,
                                   ri, 16, 16);
            T *tm = S.Tm + 256 * jb;
            mf::tile_for<T>(0, 0, [&](int r, int i, int j) { tm[i * 16 + j] = acc[r]; });
            wave_gfence();
            acc = blk16<false>(mf::zero4<T>(), Li + (int64_t)16 * ib * m + 16 * ib, m, tm, 16, ri, ri, 16);
            mf::tile_for<T>(0, 0, [&](int r, int i, int j) {
                if (i < ri) Li[(int64_t)(16 * ib + i) * m + 16 * jb + j] = -acc[r];
            });
        }
        __syncthreads();
    }
    for (int e = tid; e < m * m; e += nthr()) {
        const int i = e / m, j = e - (e / m) * m;
        const T v = j <= i ? Li[e] : T(0);
        Li[e] = v;
        S.LiT[(int64_t)j * m + i] = v;
    }
    __syncthreads();
}

// Where a pass's per-stage factors go.
// Leaf records (LeafRec layout, element type T): up or down record of stage s.
template <class T>
struct LeafOut {
    T *base;
    int n, m;
    bool up;
    __device__ T *at(int s) const {
        const LeafRec R{n, m};
        return base + (int64_t)s * R.per_stage() + (up ? 0 : R.up());
    }
    __device__ void P(int s, int i, int j, T v) const { at(s)[LeafRec{n, m}.P() + i * n + j] = v; }
    __device__ void K(int s, int i, int j, T v) const { at(s)[LeafRec{n, m}.K() + i * n + j] = v; }
    __device__ void V(int s, int i, int j, T v) const { at(s)[LeafRec{n, m}.V() + i * n + j] = v; }
    __device__ void Lt(int s, int i, int j, T v) const { at(s)[LeafRec{n, m}.Lt() + i * n + j] = v; }
    // the records of stage s that the products write (row length n)
    __device__ T *Prec(int s) const { return at(s) + LeafRec{n, m}.P(); }
    __device__ T *Krec(int s) const { return at(s) + LeafRec{n, m}.K(); }
    __device__ T *Vrec(int s) const { return up ? at(s) + LeafRec{n, m}.V() : nullptr; }
    __device__ T *Ltrec(int s) const { return up ? at(s) + LeafRec{n, m}.Lt() : nullptr; }
    __device__ void L(int s, const T *Li, const T *LiT) const {
        T *d = at(s);
        const LeafRec R{n, m};
        for (int e = threadIdx.x; e < m * m; e += nthr()) {
            d[R.L() + e] = Li[e];
            d[R.LT() + e] = LiT[e];
        }
    }
};

// Master-slot factors (SlotLayout): up pass uK, uP, uV, uL, uLT (and, for
// the superposition sweep, L_t in the dL place); down pass K, dL, dLT.
struct SlotOut {
    double *slots;
    int first, n;
    bool up;
    bool lt;
    __device__ double *at(int s) const { return slots + (int64_t)(first + s) * SlotLayout{n}.size(); }
    __device__ void P(int s, int i, int j, double v) const {
        if (up) at(s)[SlotLayout{n}.uP() + i * n + j] = v;
    }
    __device__ void K(int s, int i, int j, double v) const {
        const SlotLayout L{n};
        at(s)[(up ? L.uK() : L.K()) + i * n + j] = v;
    }
    __device__ void V(int s, int i, int j, double v) const {
        if (up) at(s)[SlotLayout{n}.uV() + i * n + j] = v;
    }
    __device__ void Lt(int s, int i, int j, double v) const {
        if (lt) at(s)[SlotLayout{n}.dL() + i * n + j] = v;
    }
    // the records of stage s that the products write (row length n)
    __device__ double *Prec(int s) const { return up ? at(s) + SlotLayout{n}.uP() : nullptr; }
    __device__ double *Krec(int s) const { return at(s) + (up ? SlotLayout{n}.uK() : SlotLayout{n}.K()); }
    __device__ double *Vrec(int s) const { return up ? at(s) + SlotLayout{n}.uV() : nullptr; }
    __device__ double *Ltrec(int s) const { return lt ? at(s) + SlotLayout{n}.dL() : nullptr; }
    __device__ void L(int s, const double *Li, const double *LiT) const {
        double *d = at(s);
        const SlotLayout SL{n};
        const int oL = up ? SL.uL() : SL.dL(), oT = up ? SL.uLT() : SL.dLT();
        for (int e = threadIdx.x; e < n * n; e += nthr()) {
            d[oL + e] = Li[e];
            d[oT + e] = LiT[e];
        }
    }
};

// [A B] of a stage into the workspace (n x (n + m), row-major, element
// type T), eight loads per thread in flight before their stores (a load
// issued after a store to memory the compiler cannot tell apart waits for
// it).
template <class T>
__device__ __forceinline__ void load_ab(WS<T> &S, const StageSrc &src) {
    const int n = S.n, m = S.m, nw = S.nw, total = n * nw, nt = nthr();
    for (int e0 = threadIdx.x; e0 < total; e0 += 8 * nt) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * nt, i = e / nw, j = e - (e / nw) * nw;
            v[u] = e < total ? (T)(j < n ? src.A[(int64_t)i * n + j] : src.B[(int64_t)i * m + j - n]) : T(0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (e0 + u * nt < total) S.AB[e0 + u * nt] = v[u];
    }
}

// Backward pass over `count` stages (local s = count-1 .. 0), matrix lines
// only.  RED: Alg. 4 (state P, V, Q_w_hat in the workspace); otherwise Alg. 1
// from the P in the workspace.  pre(s) runs before stage s and sees P_{s+1}.
// BF: P [A B], A'W_A, A'W_B and B'W_B (A'PA, A'PB, B'PB) on BF16 operands.
template <class T, bool RED, bool BF, class Get, class Pre, class Out>
__device__ void mpass_tile(WS<T> &S, Get get, int count, int32_t *info, int inst, int stage_base, int fail_code, Pre pre,
                      const Out &out, int *bad) {
    static_assert(!BF || sizeof(T) == 4, "BF16 products accumulate in FP32");
    const int n = S.n, m = S.m, nw = S.nw, tid = threadIdx.x;
    count = uni(count);
    for (int s = count - 1; s >= 0; --s) {
        pre(s);
        const StageSrc src = get(s);
        for (int e = tid; e < n * nw; e += nthr()) {
            const int i = e / nw, j = e - (e / nw) * nw;
            S.AB[e] = (T)(j < n ? src.A[(int64_t)i * n + j] : src.B[(int64_t)i * m + j - n]);
        }
        __syncthreads();
        // W = P [A B]; Alg. 4: B'V, A'V
        gemm_big<BF, false, false>(n, nw, n, S.P, n, S.AB, nw, false,
                                   [&](int i, int j, T c) { S.W[(int64_t)i * nw + j] = c; });
        if constexpr (RED) {
            gemm_tile<true, false>(m, n, n, S.AB + n, nw, S.V, n, false,
                              [&](int i, int j, T c) { S.BV[(int64_t)i * n + j] = c; });
            gemm_tile<true, false>(n, n, n, S.AB, nw, S.V, n, false, [&](int i, int j, T c) { S.AV[(int64_t)i * n + j] = c; });
        }
        __syncthreads();
        // F = Qx + A'W_A (symmetric), H = Qxw + A'W_B, G = Qw + B'W_B (symmetric)
        gemm_big<BF, true, false>(n, n, n, S.AB, nw, S.W, nw, true, [&](int i, int j, T c) {
            if (i >= j) {
                const T v = (T)src.Qx[(int64_t)i * n + j] + c;
                S.F[(int64_t)i * n + j] = v;
                S.F[(int64_t)j * n + i] = v;
            }
        });
        gemm_big<BF, true, false>(n, m, n, S.AB, nw, S.W + n, nw, false, [&](int i, int j, T c) {
            S.H[(int64_t)i * m + j] = (src.Qxw ? (T)src.Qxw[(int64_t)i * m + j] : T(0)) + c;
        });
        gemm_big<BF, true, false>(m, m, n, S.AB + n, nw, S.W + n, nw, true, [&](int i, int j, T c) {
            if (i >= j) {
                const T v = (T)src.Qw[(int64_t)i * m + j] + c;
                S.G[(int64_t)i * m + j] = v;
                S.G[(int64_t)j * m + i] = v;
            }
        });
        __syncthreads();
        chol_inv(S, m, bad);
        if (tid == 0 && *bad) {
            record_failure(info, inst, fail_code, stage_base < 0 ? -1 : stage_base + s);
            *bad = 0;
        }
        out.L(s, S.Li, S.LiT);
        // Y' = H L^{-T}; Alg. 4: X = L^{-1} B'V
        gemm_tile<false, false>(n, m, m, S.H, m, S.LiT, m, false, [&](int i, int j, T c) { S.HY[(int64_t)i * m + j] = c; });
        if constexpr (RED) {
            gemm_tile<false, false>(m, n, m, S.Li, m, S.BV, n, false, [&](int i, int j, T c) { S.X[(int64_t)i * n + j] = c; });
        }
        __syncthreads();
        // P = F - Y'Y (symmetric), K = -L^{-T} Y
        gemm_tile<false, true>(n, n, m, S.HY, m, S.HY, m, true, [&](int i, int j, T c) {
            if (i >= j) {
                const T v = S.F[(int64_t)i * n + j] - c;
                S.P[(int64_t)i * n + j] = v;
                S.P[(int64_t)j * n + i] = v;
                out.P(s, i, j, v);
                out.P(s, j, i, v);
            }
        });
        gemm_tile<false, true>(m, n, m, S.LiT, m, S.HY, m, false, [&](int i, int j, T c) { out.K(s, i, j, -c); });
        if constexpr (RED) {
            // Q_w_hat += X'X, V = A'V - Y'X, L_t = -L^{-T} X
            gemm_tile<true, false>(n, n, m, S.X, n, S.X, n, true, [&](int i, int j, T c) {
                if (i >= j) {
                    const T v = S.Qh[(int64_t)i * n + j] + c;
                    S.Qh[(int64_t)i * n + j] = v;
                    S.Qh[(int64_t)j * n + i] = v;
                }
            });
            gemm_tile<false, false>(n, n, m, S.HY, m, S.X, n, false, [&](int i, int j, T c) {
                const T v = S.AV[(int64_t)i * n + j] - c;
                S.V[(int64_t)i * n + j] = v;
                out.V(s, i, j, v);
            });
            gemm_tile<false, false>(m, n, m, S.LiT, m, S.X, n, false, [&](int i, int j, T c) { out.Lt(s, i, j, -c); });
        }
        __syncthreads();
    }
}

// The same pass with the products on LDS panels (gemm_panel) and their
// results through epilogue descriptors: the stages with n_x > 64.
template <class T, bool RED, bool BF, class Get, class Pre, class Out>
__device__ void mpass_panel(WS<T> &S, Get get, int count, int32_t *info, int inst, int stage_base, int fail_code, Pre pre,
                      const Out &out, int *bad) {
    static_assert(!BF || sizeof(T) == 4, "BF16 products accumulate in FP32");
    const int n = S.n, m = S.m, nw = S.nw, tid = threadIdx.x;
    count = uni(count);
    for (int s = count - 1; s >= 0; --s) {
        pre(s);
        const StageSrc src = get(s);
        load_ab(S, src);
        __syncthreads();
        // W = P [A B]; Alg. 4: B'V, A'V
        gemm_big_panel<BF, false, false>(n, nw, n, S.P, n, S.AB, nw, false, to(S.W, nw));
        if constexpr (RED) {
            gemm_panel<true, false>(m, n, n, S.AB + n, nw, S.V, n, false, to(S.BV, n));
            gemm_panel<true, false>(n, n, n, S.AB, nw, S.V, n, false, to(S.AV, n));
        }
        __syncthreads();
        // F = Qx + A'W_A (symmetric), H = Qxw + A'W_B, G = Qw + B'W_B (symmetric)
        {
            Ep<T> e = to(S.F, n);
            e.D64 = src.Qx;
            e.ldd = n;
            e.sym = true;
            gemm_big_panel<BF, true, false>(n, n, n, S.AB, nw, S.W, nw, true, e);
        }
        {
            Ep<T> e = to(S.H, m);
            e.D64 = src.Qxw;
            e.ldd = m;
            gemm_big_panel<BF, true, false>(n, m, n, S.AB, nw, S.W + n, nw, false, e);
        }
        {
            Ep<T> e = to(S.G, m);
            e.D64 = src.Qw;
            e.ldd = m;
            e.sym = true;
            gemm_big_panel<BF, true, false>(m, m, n, S.AB + n, nw, S.W + n, nw, true, e);
        }
        __syncthreads();
        chol_inv(S, m, bad);
        if (tid == 0 && *bad) {
            record_failure(info, inst, fail_code, stage_base < 0 ? -1 : stage_base + s);
            *bad = 0;
        }
        out.L(s, S.Li, S.LiT);
        // Y' = H L^{-T}; Alg. 4: X = L^{-1} B'V
        gemm_panel<false, false>(n, m, m, S.H, m, S.LiT, m, false, to(S.HY, m));
        if constexpr (RED) gemm_panel<false, false>(m, n, m, S.Li, m, S.BV, n, false, to(S.X, n));
        __syncthreads();
        // P = F - Y'Y (symmetric), K = -L^{-T} Y
        {
            Ep<T> e = to(S.P, n);
            e.DT = S.F;
            e.ldd = n;
            e.sgn = T(-1);
            e.sym = true;
            e.R = out.Prec(s);
            e.ldr = n;
            gemm_panel<false, true>(n, n, m, S.HY, m, S.HY, m, true, e);
        }
        {
            Ep<T> e = to(out.Krec(s), n);
            e.sgn = T(-1);
            gemm_panel<false, true>(m, n, m, S.LiT, m, S.HY, m, false, e);
        }
        if constexpr (RED) {
            // Q_w_hat += X'X, V = A'V - Y'X, L_t = -L^{-T} X
            {
                Ep<T> e = to(S.Qh, n);
                e.DT = S.Qh;
                e.ldd = n;
                e.sym = true;
                gemm_panel<true, false>(n, n, m, S.X, n, S.X, n, true, e);
            }
            {
                Ep<T> e = to(S.V, n);
                e.DT = S.AV;
                e.ldd = n;
                e.sgn = T(-1);
                e.R = out.Vrec(s);
                e.ldr = n;
                gemm_panel<false, false>(n, n, m, S.HY, m, S.X, n, false, e);
            }
            {
                Ep<T> e = to(out.Ltrec(s), n);
                e.sgn = T(-1);
                gemm_panel<false, false>(m, n, m, S.LiT, m, S.X, n, false, e);
            }
        }
        __syncthreads();
    }
}

// A pass over `count` stages: LDS-panel products out of line for the large
// stages (BIG: n_x > 64), the inline per-tile products otherwise.
template <class T, bool RED, bool BF, bool BIG, class Get, class Pre, class Out>
__device__ __forceinline__ void mpass(WS<T> &S, Get get, int count, int32_t *info, int inst, int stage_base,
                                      int fail_code, Pre pre, const Out &out, int *bad) {
    if constexpr (BIG)
        mpass_panel<T, RED, BF>(S, get, count, info, inst, stage_base, fail_code, pre, out, bad);
    else
        mpass_tile<T, RED, BF>(S, get, count, info, inst, stage_base, fail_code, pre, out, bad);
}

__device__ __forceinline__ StageSrc leaf_stage(const DevProb &p, int t) { return prob_stage(p, t); }

// Start of Alg. 4: P = 0, V = I, Q_w_hat = 0.
template <class T>
__device__ void init_red(WS<T> &S) {
    const int n = S.n;
    for (int e = threadIdx.x; e < n * n; e += nthr()) {
        S.P[e] = T(0);
        S.V[e] = (e / n == e % n) ? T(1) : T(0);
        S.Qh[e] = T(0);
    }
    __syncthreads();
}

template <class T>
__device__ T *unit_ws(const GroupArgs &g) {
    return reinterpret_cast<T *>(static_cast<char *>(g.lbw) + (int64_t)blockIdx.x * g.lbw_unit);
}

// ------------------------------------------------------------ matrix side
template <class T, bool BF, bool BIG>
__global__ void __launch_bounds__(LB_MT) kl_leaf_up(GroupArgs g) {
    __shared__ int bad;
    const int n = g.nx, m = g.nu, tid = threadIdx.x;
    WS<T> S;
    S.bind(unit_ws<T>(g), n, m);
    if (tid == 0) bad = 0;
    const SlotLayout SL{n};
    for (int li = blockIdx.x; li < g.nleaves; li += gridDim.x) {
        const LeafItem it = sv::load_leaf(g.leaves, li);
        if ((it.flags & LEAF_TOP) || inst_skipped(g.probs, it.inst)) continue;
        const DevProb p = load_prob(g.probs, it.inst);
        double *out = g.slots + (int64_t)it.slot * SL.size();
        if (it.flags & LEAF_REUSE) {
            // stored factorization current (receding-horizon plans): only its
            // cached M1 goes to this call's slot
            const double *c = g.m1cache + (int64_t)it.m1 * 3 * n * n;
            for (int e = tid; e < 3 * n * n; e += nthr()) out[e] = c[e];
            continue;
        }
        double *cache = (g.m1cache && it.m1 >= 0) ? g.m1cache + (int64_t)it.m1 * 3 * n * n : nullptr;
        T *base = reinterpret_cast<T *>(g.fstore) + g.rec_stage(it.scratch) * (int64_t)LeafRec{n, m}.per_stage();
        auto get = [&](int s) { return leaf_stage(p, it.t0 + s); };
        const LeafOut<T> o{base, n, m, true};
        if (!(it.flags & LEAF_LAST)) {
            init_red(S);
            mpass<T, true, BF, BIG>(S, get, it.len, g.info, it.inst, it.t0, 2, [](int) {}, o, &bad);
            for (int e = tid; e < n * n; e += nthr()) {
                const int i = e / n, j = e % n;
                const double a = (double)S.V[(int64_t)j * n + i], q = (double)S.Qh[e], x = (double)S.P[e];
                out[SL.A() + e] = a;
                if (!g.ident) out[SL.Qw() + e] = q;
                out[SL.Qx() + e] = x;
                if (cache) {
                    cache[SL.A() + e] = a;
                    if (!g.ident) cache[SL.Qw() + e] = q;
                    cache[SL.Qx() + e] = x;
                }
            }
            if (g.ident) rank_reveal(S.Qh, n, unit_roundoff<T>(), out + SL.Qw(), cache ? cache + SL.Qw() : nullptr);
        } else {
            for (int e = tid; e < n * n; e += nthr()) S.P[e] = (T)p.QxN[e];
            __syncthreads();
            mpass<T, false, BF, BIG>(S, get, it.len, g.info, it.inst, it.t0, 2, [](int) {}, o, &bad);
            for (int e = tid; e < n * n; e += nthr()) out[SL.Qx() + e] = (double)S.P[e];
        }
        __syncthreads();
    }
}

template <class T, bool BF, bool BIG>
__global__ void __launch_bounds__(LB_MT) kl_leaf_down(GroupArgs g) {
    __shared__ int bad;
    const int n = g.nx, m = g.nu, tid = threadIdx.x;
    WS<T> S;
    S.bind(unit_ws<T>(g), n, m);
    if (tid == 0) bad = 0;
    for (int li = blockIdx.x; li < g.nleaves; li += gridDim.x) {
        const LeafItem it = sv::load_leaf(g.leaves, li);
        // only whole-problem leaves need the factorization with the true
        // terminal; the others are solved from their up records
        if (!(it.flags & LEAF_TOP) || inst_skipped(g.probs, it.inst)) continue;
        const DevProb p = load_prob(g.probs, it.inst);
        T *base = reinterpret_cast<T *>(g.fstore) + g.rec_stage(it.scratch) * (int64_t)LeafRec{n, m}.per_stage();
        for (int e = tid; e < n * n; e += nthr()) S.P[e] = (T)p.QxN[e];
        __syncthreads();
        auto get = [&](int s) { return leaf_stage(p, it.t0 + s); };
        mpass<T, false, BF, BIG>(S, get, it.len, g.info, it.inst, it.t0, 2, [](int) {}, LeafOut<T>{base, n, m, false},
                            &bad);
        __syncthreads();
    }
}

// Waits (thread 0) until the items this one depends on carry the current
// epoch; a bounded wait records a failure instead of hanging.
__device__ void wait_deps(const GroupArgs &g, const TreeItem &it) {
    if (threadIdx.x == 0) {
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
}

__device__ void publish(const GroupArgs &g, int idx) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(&g.flags[idx], g.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
}

template <bool BIG>
__global__ void __launch_bounds__(LB_MT) kl_tree(GroupArgs g) {
    __shared__ int s_item, bad;
    const int n = g.nx, tid = threadIdx.x;
    const SlotLayout SL{n};
    WS<double> S;
    S.bind(unit_ws<double>(g), n, n);
    if (tid == 0) bad = 0;
    double *slots = g.slots;
    auto slot = [&](int s) { return slots + (int64_t)s * SL.size(); };
    for (;;) {
        if (tid == 0) s_item = atomicAdd(g.queue, 1);
        __syncthreads();
        const int idx = uni(s_item);
        __syncthreads();
        if (idx >= g.nitems) break;
        const TreeItem it = load_item(g.items, idx);
        wait_deps(g, it);
        auto get = [&](int s) { return slot_stage(slot(it.first + s), n, g.ident); };
        if (inst_skipped(g.probs, it.inst)) {
            // excluded instance: only its completion flag is published
        } else if (it.kind == ITEM_UP) {
            init_red(S);
            mpass<double, true, false, BIG>(S, get, it.count, g.info, it.inst, -1, 3, [](int) {},
                                       SlotOut{slots, it.first, n, true, g.superpose != 0}, &bad);
            double *out = slot(it.out_slot);
            for (int e = tid; e < n * n; e += nthr()) {
                const int i = e / n, j = e % n;
                out[SL.A() + e] = S.V[(int64_t)j * n + i];
                if (!g.ident) out[SL.Qw() + e] = S.Qh[e];
                out[SL.Qx() + e] = S.P[e];
            }
            if (g.ident) rank_reveal(S.Qh, n, unit_roundoff<double>(), out + SL.Qw(), nullptr);
        } else if (it.kind == ITEM_DOWN && g.superpose) {
            // solved by the vector pass from the up records: nothing to factor
        } else {
            // Alg. 1 on the master stages from the true terminal (a level's
            // last item, up records) or from the parent's message (down
            // records; top, and below it without superposition)
            const bool upl = it.kind == ITEM_UP_LAST;
            const double *msg = it.kind == ITEM_DOWN ? slot(it.out_slot) : nullptr;
            double *term = it.last ? slot(it.term_slot) : nullptr;
            for (int e = tid; e < n * n; e += nthr()) S.P[e] = term ? term[SL.Qx() + e] : msg[SL.P() + e];
            __syncthreads();
            mpass<double, false, false, BIG>(
                S, get, it.count, g.info, it.inst, -1, 3,
                [&](int s) {      // M2 for child s: P at the end of master stage s
                    if (!upl) {
                        double *d = slot(it.first + s) + SL.P();
                        for (int e = tid; e < n * n; e += nthr()) d[e] = S.P[e];
                    }
                },
                SlotOut{slots, it.first, n, upl, false}, &bad);
            // a level's last item: its reduced terminal; the top: P_0, for the optimal value
            double *d = upl ? slot(it.out_slot) + SL.Qx() : it.kind == ITEM_TOP ? term + SL.P() : nullptr;
            if (d)
                for (int e = tid; e < n * n; e += nthr()) d[e] = S.P[e];
        }
        publish(g, idx);
    }
}

// ------------------------------------------------------------ vector side
constexpr int VMAX = 128;
// threads of the vector-line kernels, at most (8 wavefronts; the launch
// takes 4 or 8, and every loop and partition below follows the launch): with
// 8, a matrix-vector product of up to 128 rows takes two passes of 64 rows
// (row form) or eight column groups (column form), so its loads are in
// flight in few round trips
constexpr int VNT = 512;

struct VS {
    double Psi[VMAX], pt[VMAX], av[VMAX], d[VMAX], x[VMAX], gw[VMAX], z[VMAX], kk[VMAX], wv[VMAX], v[VMAX],
        lamN[VMAX], y[VMAX];
    double red[VNT / 64];
    double gred[VNT];
};

__device__ __forceinline__ double block_sum(double v, VS &S) {
    v = sv::wave_sum(v);
    __syncthreads();
    if (lane() == 0) S.red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < nwav(); ++w) s += S.red[w];
    return s;
}

// y(i) = sum_k op(M)(i,k) x[k] for i < R, k < C (R, C <= 128), handed to
// out(i, y) by one thread per i; every thread of the workgroup must call it.
// COLUMN-read form op(M)(i,k) = M[k*ld+i]: output i and a contiguous part of
// the k range per thread (consecutive threads on consecutive words), the
// parts summed in a fixed order through LDS.  ROW-read form
// op(M)(i,k) = M[i*ld+k]: 16 lanes per output row, strided over k, summed
// with lane shuffles.  Several loads per thread are in flight in both.
template <bool ROW, class U, class Out>
__device__ __forceinline__ void gemv(const U *M, int ld, const double *x, int R, int C, Out out, double *red) {
    const int tid = threadIdx.x;
    if constexpr (!ROW) {
        int Rp = 16;
        while (Rp < R) Rp <<= 1;
        const int parts = nthr() / Rp, i = tid & (Rp - 1), p = tid / Rp;
        const int chunk = (C + parts - 1) / parts, k0 = p * chunk, k1 = k0 + chunk < C ? k0 + chunk : C;
        double acc = 0.0;
        if (M && i < R) {
#pragma unroll 8
            for (int k = k0; k < k1; ++k) acc += (double)M[(int64_t)k * ld + i] * x[k];
        }
        red[tid] = acc;
        __syncthreads();
        if (tid < R) {
            double s = 0.0;
            for (int q = 0; q < parts; ++q) s += red[q * Rp + tid];
            out(tid, s);
        }
        __syncthreads();
    } else {
        const int l = lane(), c16 = l & 15, row = wave() * 4 + (l >> 4);
        for (int base = 0; base < R; base += nthr() / 16) {
            const int i = base + row;
            double acc = 0.0;
            if (M && i < R) {
#pragma unroll 8
                for (int k = c16; k < C; k += 16) acc += (double)M[(int64_t)i * ld + k] * x[k];
            }
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
            if (c16 == 0 && i < R) out(i, acc);
        }
    }
}

// Both products of one row-major matrix M (rows x cols, leading dimension
// ld) from a single read: M'v (outputs i < cols, handed to ocol(i, y)) and
// M u (outputs k < rows, handed to orow(k, y)).  The threads form groups of
// G = cols rounded up to a power of two (16, 32 or 64, inside one
// wavefront); thread i of group p reads M(k, i) for the rows k of the
// group's chunk, adds M(k, i) v_k to its column sum and passes M(k, i) u_i
// through a DPP sum over the group for the row sum of k.  Every group runs
// the same number of iterations, so the sums run with all lanes active.
// The column sums of the groups are added through LDS (red, VNT doubles) in a
// fixed order; all threads of the workgroup must call it.
template <int G, class OC, class OR>
__device__ __forceinline__ void gemv_dual(const double *M, int ld, const double *v, const double *u, int rows,
                                          int cols, OC ocol, OR orow, double *red) {
    const int tid = threadIdx.x, parts = nthr() / G, i = tid & (G - 1), p = tid / G;
    const int chunk = (rows + parts - 1) / parts, k0 = p * chunk;
    const bool col = i < cols;
    const double ui = col ? u[i] : 0.0;
    double acc = 0.0;
#pragma unroll 8
    for (int q = 0; q < chunk; ++q) {
        const int k = k0 + q;
        const bool ok = col && k < rows;
        const double mk = ok ? M[(int64_t)k * ld + i] : 0.0;
        acc += ok ? mk * v[k] : 0.0;
        const double r = sv::group_sum<G>(mk * ui);
        if (i == 0 && k < rows) orow(k, r);
    }
    red[tid] = acc;
    __syncthreads();
    if (tid < cols) {
        double s = 0.0;
        for (int q = 0; q < parts; ++q) s += red[q * G + tid];
        ocol(tid, s);
    }
    __syncthreads();
}

// gemv_dual for any cols <= 64; larger matrices take the two reads of gemv.
template <class OC, class OR>
__device__ __forceinline__ void gemv_both(const double *M, int ld, const double *v, const double *u, int rows,
                                          int cols, OC ocol, OR orow, double *red) {
    if (cols <= 16)
        gemv_dual<16>(M, ld, v, u, rows, cols, ocol, orow, red);
    else if (cols <= 32)
        gemv_dual<32>(M, ld, v, u, rows, cols, ocol, orow, red);
    else if (cols <= 64)
        gemv_dual<64>(M, ld, v, u, rows, cols, ocol, orow, red);
    else {
        gemv<false>(M, ld, v, cols, rows, ocol, red);
        gemv<true>(M, ld, u, rows, cols, orow, red);
    }
}

// Operands of one backward stage of the vector recursion (as in the
// register-resident kernels): P_{t+1} (TR-typed record, FP64 terminal or
// message, or zero), V_{t+1} (record or identity), L^{-1}, L^{-T}, K.
template <class TR>
struct VSrcL {
    const TR *Pn;
    const double *Pn64;
    const TR *Vn;
    const TR *Li, *LT, *K;
    const double *A, *B, *a, *lx, *lw;
    double c;
};

// One backward stage: P a, pt = Psi - P a, cbar += 1/2 a'Pa - Psi'a + c,
// g_w = B' pt - l_w, z = L^{-1} g_w, Psi_t = A' pt + K' g_w - l_x,
// cbar -= z'z / 2, k = L^{-T} z; Alg. 4: v += V_{t+1}' (a + B k).
// cbar lives in thread 0.  Psi_t and k are left in S.Psi and S.kk.
template <bool RED, bool WANTK, class TR>
__device__ void vstage(VS &S, const VSrcL<TR> &q, int n, int m, double &cbar) {
    const int tid = threadIdx.x;
    for (int i = tid; i < n; i += nthr()) S.av[i] = q.a ? q.a[i] : 0.0;
    __syncthreads();
    double part = 0.0;
    if (q.Pn)
        gemv<false>(q.Pn, n, S.av, n, n, [&](int i, double pa) {
            S.pt[i] = S.Psi[i] - pa;
            part += S.av[i] * (0.5 * pa - S.Psi[i]);
        }, S.gred);
    else
        gemv<false>(q.Pn64, n, S.av, n, n, [&](int i, double pa) {
            S.pt[i] = S.Psi[i] - pa;
            part += S.av[i] * (0.5 * pa - S.Psi[i]);
        }, S.gred);
    const double s1 = block_sum(part, S);
    if (tid == 0) cbar += s1 + q.c;
    gemv<false>(q.B, m, S.pt, m, n, [&](int j, double v) { S.gw[j] = v - (q.lw ? q.lw[j] : 0.0); }, S.gred);
    __syncthreads();
    double zz = 0.0;
    gemv<false>(q.LT, m, S.gw, m, m, [&](int i, double v) {
        S.z[i] = v;
        zz += v * v;
    }, S.gred);
    gemv<false>(q.A, n, S.pt, n, n, [&](int i, double v) { S.y[i] = v - (q.lx ? q.lx[i] : 0.0); }, S.gred);
    __syncthreads();
    gemv<false>(q.K, n, S.gw, n, m, [&](int i, double v) { S.Psi[i] = S.y[i] + v; }, S.gred);
    const double s2 = block_sum(zz, S);
    if (tid == 0) cbar -= 0.5 * s2;
    if constexpr (RED || WANTK) {
        gemv<false>(q.Li, m, S.z, m, m, [&](int i, double v) { S.kk[i] = v; }, S.gred);
        __syncthreads();
    }
    if constexpr (RED) {
        gemv<true>(q.B, m, S.kk, n, m, [&](int i, double v) { S.d[i] = S.av[i] + v; }, S.gred);
        __syncthreads();
        if (q.Vn)
            gemv<false>(q.Vn, n, S.d, n, n, [&](int i, double v) { S.v[i] += v; }, S.gred);
        else
            for (int i = tid; i < n; i += nthr()) S.v[i] += S.d[i];
        __syncthreads();
    }
}

// One forward stage (Alg. 3): w = K x + k (+ L lam_N), x_{t+1} = A x + a + B w
// and lam_t = P_t x - Psi_t (+ V_t lam_N); x, w, lam of stage t written to
// the outputs when given.
template <class TR>
__device__ __forceinline__ void fstage(VS &S, int n, int m, const TR *K, const double *kvec, const TR *Lt,
                                       const double *A, const double *B, const double *a, const TR *P,
                                       const double *Psi, const TR *Vt, double *x_out, double *w_out,
                                       double *lam_out) {
    const int tid = threadIdx.x;
    for (int i = tid; i < n; i += nthr())
        if (x_out) x_out[i] = S.x[i];
    gemv<true>(K, n, S.x, m, n, [&](int i, double v) { S.wv[i] = v + kvec[i]; }, S.gred);
    gemv<true>(A, n, S.x, n, n, [&](int i, double v) { S.y[i] = v + (a ? a[i] : 0.0); }, S.gred);
    if (P) gemv<false>(P, n, S.x, n, n, [&](int i, double v) { S.d[i] = v - Psi[i]; }, S.gred);
    __syncthreads();
    if (Lt) {
        gemv<true>(Lt, n, S.lamN, m, n, [&](int i, double v) { S.wv[i] += v; }, S.gred);
        gemv<true>(Vt, n, S.lamN, n, n, [&](int i, double v) { S.d[i] += v; }, S.gred);
        __syncthreads();
    }
    for (int i = tid; i < m; i += nthr())
        if (w_out) w_out[i] = S.wv[i];
    for (int i = tid; i < n; i += nthr())
        if (lam_out) lam_out[i] = S.d[i];
    gemv<true>(B, m, S.wv, n, m, [&](int i, double v) { S.y[i] += v; }, S.gred);
    __syncthreads();
    for (int i = tid; i < n; i += nthr()) S.x[i] = S.y[i];
    __syncthreads();
}

// 1/2 x'Px - Psi'x + cbar at the x in S.x (result in thread 0).
template <class TP>
__device__ double cost_to_go(VS &S, const TP *P, int n, double cbar) {
    double part = 0.0;
    gemv<false>(P, n, S.x, n, n, [&](int i, double v) { part += S.x[i] * (0.5 * v - S.Psi[i]); }, S.gred);
    const double s = block_sum(part, S);
    return s + cbar;
}

template <class TR>
__device__ VSrcL<TR> prob_src(const sv::Prob &p, int t) {
    VSrcL<TR> q;
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

__device__ VSrcL<double> slot_src(const double *sl, int n) {
    const SlotLayout L{n};
    VSrcL<double> q;
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

template <class TR>
__global__ void __launch_bounds__(VNT) kw_leaf_up(GroupArgs g) {
    __shared__ VS S;
    if (sv::pass_idle(g)) return;
    const int n = g.nx, m = g.nu, tid = threadIdx.x;
    const LeafItem it = sv::load_leaf(g.leaves, blockIdx.x);
    if ((it.flags & LEAF_TOP) || sv::skip_inst(g, it.inst)) return;
    const sv::Prob p = sv::load_prob(g.probs, it.inst);
    const LeafRec R{n, m};
    const SlotLayout SL{n};
    const TR *rec = reinterpret_cast<const TR *>(g.fstore) + g.rec_stage(it.scratch) * (int64_t)R.per_stage();
    double *out = g.slots + (int64_t)it.slot * SL.size();
    const bool last = (it.flags & LEAF_LAST) != 0;
    for (int i = tid; i < n; i += nthr()) {
        S.Psi[i] = (last && p.lN) ? -p.lN[i] : 0.0;
        S.v[i] = 0.0;
    }
    double cbar = (last && p.cN) ? p.cN[0] : 0.0;
    double *vec0 = g.fvec + g.rec_stage(it.scratch) * (int64_t)R.vec();
    __syncthreads();
    for (int s = uni(it.len) - 1; s >= 0; --s) {
        VSrcL<TR> q = prob_src<TR>(p, it.t0 + s);
        const TR *r = rec + (int64_t)s * R.per_stage();
        const TR *rn = r + R.per_stage();
        const bool end = s + 1 == it.len;
        q.Li = r + R.L();
        q.LT = r + R.LT();
        q.K = r + R.K();
        q.Pn = end ? nullptr : rn + R.P();
        if (!last) {
            q.Vn = end ? nullptr : rn + R.V();
            vstage<true, false>(S, q, n, m, cbar);
        } else {
            q.Pn64 = end ? p.QxN : nullptr;
            vstage<false, true>(S, q, n, m, cbar);
        }
        // Psi_t and k_{t+1} of this sweep, for the leaf solve
        double *vec = vec0 + (int64_t)s * R.vec();
        for (int i = tid; i < n; i += nthr()) vec[i] = S.Psi[i];
        for (int i = tid; i < m; i += nthr()) vec[n + i] = S.kk[i];
        __syncthreads();
    }
    for (int i = tid; i < n; i += nthr()) {
        if (!last) out[SL.a() + i] = S.v[i];
        out[SL.lx() + i] = -S.Psi[i];
    }
    if (tid == 0) out[SL.c()] = cbar;
}

// Leaf solve from the stored preliminary solution (superposition in the
// terminal costate lam_N = P_hat x_hat_{i+1} - Psi_hat, since Psi and k are
// affine in the terminal linear term):
//   w_t = K x_t + k_0 + L lam_N,  lam_t = P_t x_t - Psi_0,t + V_t lam_N.
// The last leaf was reduced with the true terminal (no lam_N terms).
template <class TR>
__device__ void leaf_forward(VS &S, const GroupArgs &g, const sv::Prob &p, const LeafItem &it) {
    const int n = g.nx, m = g.nu, tid = threadIdx.x;
    const LeafRec R{n, m};
    const SlotLayout SL{n};
    const int64_t stage0 = g.rec_stage(it.scratch);
    const TR *rec = reinterpret_cast<const TR *>(g.fstore) + stage0 * (int64_t)R.per_stage();
    const double *vec0 = g.fvec + stage0 * (int64_t)R.vec();
    const double *msg = g.slots + (int64_t)it.slot * SL.size();
    const bool last = (it.flags & LEAF_LAST) != 0;
    if (!last && g.superpose) {
        for (int i = tid; i < n; i += nthr()) S.lamN[i] = msg[SL.lamN() + i];    // sent by the master level
    } else if (!last) {
        const double *nxt = msg + SL.size();           // the next leaf's slot: x_hat_{i+1}
        for (int i = tid; i < n; i += nthr()) S.x[i] = nxt[SL.xh() + i];
        __syncthreads();
        gemv<false>(msg + SL.P(), n, S.x, n, n, [&](int i, double v) { S.lamN[i] = v - msg[SL.Psi() + i]; }, S.gred);
        __syncthreads();
    }
    for (int i = tid; i < n; i += nthr()) S.x[i] = msg[SL.xh() + i];
    __syncthreads();
    const int len = uni(it.len);
    for (int s = 0; s < len; ++s) {
        const int t = it.t0 + s;
        const TR *r = rec + (int64_t)s * R.per_stage();
        const double *vec = vec0 + (int64_t)s * R.vec();
        fstage<TR>(S, n, m, r + R.K(), vec + n, last ? nullptr : r + R.Lt(), p.A + (int64_t)t * p.sA,
                   p.B + (int64_t)t * p.sB, p.a ? p.a + (int64_t)t * p.sa : nullptr, r + R.P(), vec,
                   last ? nullptr : r + R.V(), p.x + (int64_t)t * n, p.w + (int64_t)t * m, p.lam + (int64_t)t * n);
    }
    if (last) {
        const int64_t t = it.t0 + len;
        gemv<false>(p.QxN, n, S.x, n, n, [&](int i, double v) {
            p.lam[t * n + i] = v + (p.lN ? p.lN[i] : 0.0);     // lam_N = QxN x_N + lN
            p.x[t * n + i] = S.x[i];
        }, S.gred);
    }
}

template <class TR>
__global__ void __launch_bounds__(VNT) kw_leaf_down(GroupArgs g) {
    __shared__ VS S;
    if (sv::pass_idle(g)) return;
    const int n = g.nx, m = g.nu, tid = threadIdx.x;
    const LeafItem it = sv::load_leaf(g.leaves, blockIdx.x);
    if (sv::skip_inst(g, it.inst)) return;
    const sv::Prob p = sv::load_prob(g.probs, it.inst);
    if (!(it.flags & LEAF_TOP)) {
        leaf_forward<TR>(S, g, p, it);
        return;
    }
    // whole-problem leaf: vector part of Alg. 1-2 with the true terminal on
    // the down records, then Alg. 3
    const LeafRec R{n, m};
    const int64_t stage0 = g.rec_stage(it.scratch);
    const TR *rec = reinterpret_cast<const TR *>(g.fstore) + stage0 * (int64_t)R.per_stage();
    double *vec0 = g.fvec + stage0 * (int64_t)R.vec();
    for (int i = tid; i < n; i += nthr()) {
        S.Psi[i] = p.lN ? -p.lN[i] : 0.0;
        S.x[i] = p.x0[i];
    }
    double cbar = p.cN ? p.cN[0] : 0.0;
    __syncthreads();
    const int len = uni(it.len);
    for (int s = len - 1; s >= 0; --s) {
        VSrcL<TR> q = prob_src<TR>(p, it.t0 + s);
        const TR *dn = rec + (int64_t)s * R.per_stage() + R.up();
        const bool end = s + 1 == len;
        q.Pn = end ? nullptr : dn + R.per_stage() + R.P();
        q.Pn64 = end ? p.QxN : nullptr;
        q.Li = dn + R.L();
        q.LT = dn + R.LT();
        q.K = dn + R.K();
        vstage<false, true>(S, q, n, m, cbar);
        double *vec = vec0 + (int64_t)s * R.vec();
        for (int i = tid; i < n; i += nthr()) vec[i] = S.Psi[i];
        for (int i = tid; i < m; i += nthr()) vec[n + i] = S.kk[i];
        __syncthreads();
    }
    if (p.obj) {
        const double v = cost_to_go(S, rec + R.up() + R.P(), n, cbar);
        if (tid == 0) p.obj[0] = v;
    }
    __syncthreads();
    for (int s = 0; s < len; ++s) {
        const int t = it.t0 + s;
        const TR *dn = rec + (int64_t)s * R.per_stage() + R.up();
        const double *vec = vec0 + (int64_t)s * R.vec();
        fstage<TR>(S, n, m, dn + R.K(), vec + n, nullptr, p.A + (int64_t)t * p.sA, p.B + (int64_t)t * p.sB,
                   p.a ? p.a + (int64_t)t * p.sa : nullptr, dn + R.P(), vec, nullptr, p.x + (int64_t)t * n,
                   p.w + (int64_t)t * m, p.lam + (int64_t)t * n);
    }
    const int64_t t = it.t0 + len;
    gemv<false>(p.QxN, n, S.x, n, n, [&](int i, double v) {
        p.lam[t * n + i] = v + (p.lN ? p.lN[i] : 0.0);         // lam_N = QxN x_N + lN
        p.x[t * n + i] = S.x[i];
    }, S.gred);
}

// A tree item is a chain of matrix-vector products with one workgroup per
// CU; the occupancy range of two to three waves per SIMD keeps the compiler
// from trading the loads in flight of each product's unrolled loop for
// registers.
__global__ void __launch_bounds__(VNT) __attribute__((amdgpu_waves_per_eu(2, 3))) kw_tree(GroupArgs g) {
    __shared__ VS S;
    __shared__ int s_item;
    const int n = g.nx, tid = threadIdx.x;
    const SlotLayout SL{n};
    double *slots = g.slots;
    auto slot = [&](int s) { return slots + (int64_t)s * SL.size(); };
    if (sv::pass_idle(g)) return;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(g.queue, 1);
        __syncthreads();
        const int idx = uni(s_item);
        __syncthreads();
        if (idx >= g.nitems) break;
        const TreeItem it = load_item(g.items, idx);
        wait_deps(g, it);
        const int count = it.count;
        if (sv::skip_inst(g, it.inst)) {
            // converged or excluded: nothing to do (its dependents belong to the same instance)
        } else if (it.kind == ITEM_UP) {
            // Alg. 4 on the master stages (vector lines)
            for (int i = tid; i < n; i += nthr()) {
                S.Psi[i] = 0.0;
                S.v[i] = 0.0;
            }
            double cbar = 0.0;
            __syncthreads();
            for (int s = count - 1; s >= 0; --s) {
                double *sl = slot(it.first + s);
                VSrcL<double> q = slot_src(sl, n);
                const double *sn = slot(it.first + s + 1);
                const bool end = s + 1 == count;
                q.Li = sl + SL.uL();
                q.LT = sl + SL.uLT();
                q.K = sl + SL.uK();
                q.Pn = end ? nullptr : sn + SL.uP();
                q.Vn = end ? nullptr : sn + SL.uV();
                vstage<true, false>(S, q, n, n, cbar);
                if (g.superpose) {
                    // Psi_s and k_s of this sweep, for the superposition sweep down
                    for (int i = tid; i < n; i += nthr()) {
                        sl[SL.Psi() + i] = S.Psi[i];
                        sl[SL.k() + i] = S.kk[i];
                    }
                }
                __syncthreads();
            }
            double *out = slot(it.out_slot);
            for (int i = tid; i < n; i += nthr()) {
                out[SL.a() + i] = S.v[i];
                out[SL.lx() + i] = -S.Psi[i];
            }
            if (tid == 0) out[SL.c()] = cbar;
        } else {
            // Up pass of a level's last item (Alg. 1 from the true terminal
            // on the up records), and the down pass.  Down at the top, and
            // below it without superposition: the vector part of Alg. 1 from
            // the parent's message (or the true terminal), then Alg. 3.
            // Below the top with superposition (Alg. 6, k >= 1, as in the leaf
            // solve): a forward sweep on the records of the item's up pass
            // with its terminal costate lam_N from the parent,
            //   w = K x + k_0 + L_t lam_N,  lam = P x - Psi_0 + V lam_N,
            // x+ = A_hat x + B_hat w + a_hat (no lam_N terms for the last
            // item of a level, whose records are final); child s receives
            // x_s and its terminal costate lam_{s+1}.
            const bool upl = it.kind == ITEM_UP_LAST;
            const bool top = it.kind == ITEM_TOP;
            const bool sweep = !upl && !top && g.superpose;
            const bool lterms = sweep && !it.last;
            const double *msg = upl || top ? nullptr : slot(it.out_slot);
            double *term = it.last ? slot(it.term_slot) : nullptr;
            if (sweep) {
                for (int i = tid; i < n; i += nthr()) {
                    S.x[i] = msg[SL.xh() + i];
                    S.lamN[i] = lterms ? msg[SL.lamN() + i] : 0.0;
                }
                __syncthreads();
            } else {
                const sv::Prob p = sv::load_prob(g.probs, it.inst);
                for (int i = tid; i < n; i += nthr()) {
                    S.Psi[i] = term ? -term[SL.lx() + i] : msg[SL.Psi() + i];
                    if (!upl) S.x[i] = top ? p.x0[i] : msg[SL.xh() + i];
                }
                double cbar = term ? term[SL.c()] : msg[SL.cb()];
                __syncthreads();
                for (int s = count - 1; s >= 0; --s) {
                    double *sl = slot(it.first + s);
                    VSrcL<double> q = slot_src(sl, n);
                    if (upl) {
                        q.Pn = s + 1 == count ? term + SL.Qx() : slot(it.first + s + 1) + SL.uP();
                        q.Li = sl + SL.uL();
                        q.LT = sl + SL.uLT();
                        q.K = sl + SL.uK();
                    } else {
                        // message to child s: cost to go at the end of master stage s
                        for (int i = tid; i < n; i += nthr()) sl[SL.Psi() + i] = S.Psi[i];
                        if (tid == 0) sl[SL.cb()] = cbar;
                        q.Pn = sl + SL.P();
                        q.Li = sl + SL.dL();
                        q.LT = sl + SL.dLT();
                        q.K = sl + SL.K();
                    }
                    vstage<false, true>(S, q, n, n, cbar);
                    // k_s (and for the sweep down, Psi_s of the up records)
                    if (!upl || g.superpose)
                        for (int i = tid; i < n; i += nthr()) sl[SL.k() + i] = S.kk[i];
                    if (upl && g.superpose)
                        for (int i = tid; i < n; i += nthr()) sl[SL.Psi() + i] = S.Psi[i];
                    __syncthreads();
                }
                if (upl) {
                    double *out = slot(it.out_slot);
                    for (int i = tid; i < n; i += nthr()) out[SL.lx() + i] = -S.Psi[i];
                    if (tid == 0) out[SL.c()] = cbar;
                } else if (top && p.obj) {
                    const double v = cost_to_go(S, slot(it.term_slot) + SL.P(), n, cbar);
                    if (tid == 0) p.obj[0] = v;
                }
                __syncthreads();
            }
            if (!upl) {
                for (int s = 0; s < count; ++s) {
                    double *sl = slot(it.first + s);
                    fstage<double>(S, n, n, sl + (sweep ? SL.uK() : SL.K()), sl + SL.k(),
                                   lterms ? sl + SL.dL() : nullptr, sl + SL.A(), sl + SL.Qw(), sl + SL.a(),
                                   sweep ? sl + SL.uP() : nullptr, sl + SL.Psi(), lterms ? sl + SL.uV() : nullptr,
                                   sl + SL.xh(), nullptr, sweep && s > 0 ? slot(it.first + s - 1) + SL.lamN() : nullptr);
                }
                if (it.last)
                    for (int i = tid; i < n; i += nthr()) term[SL.xh() + i] = S.x[i];
            }
            if (sweep) {
                // the last child ends where the item does: at lam_N, or for
                // the last item at the terminal node, lam = P_term x - Psi_term
                double *lend = slot(it.first + count - 1) + SL.lamN();
                if (it.last)
                    gemv<false>(term + SL.Qx(), n, S.x, n, n, [&](int i, double v) { lend[i] = v + term[SL.lx() + i]; },
                                S.gred);
                else
                    for (int i = tid; i < n; i += nthr()) lend[i] = S.lamN[i];
            } else if (top && g.superpose) {
                // terminal costate of child s, lam_{s+1} = P_{s+1} x_{s+1} -
                // Psi_{s+1}, from the cost to go sent to it and the initial
                // state of the next child (of the terminal node for the last)
                __threadfence_block();
                __syncthreads();
                for (int s = 0; s < count; ++s) {
                    double *sl = slot(it.first + s);
                    const double *xn = (s + 1 < count ? slot(it.first + s + 1) : term) + SL.xh();
                    for (int i = tid; i < n; i += nthr()) S.y[i] = xn[i];
                    __syncthreads();
                    gemv<false>(sl + SL.P(), n, S.y, n, n, [&](int i, double v) { sl[SL.lamN() + i] = v - sl[SL.Psi() + i]; },
                                S.gred);
                }
            }
        }
        publish(g, idx);
    }
}

// -------------------------------------------------------- refinement (FP64)
// Residual rho = r - K z of the KKT system of P(N) (blockwise, FP64) for the
// stages of one leaf, one stage at a time over the whole workgroup; writes
// the correction problem's data (-rho as problem data, see the register
// kernels) and the leaf's max |r|, max |rho| and objective part.
__global__ void __launch_bounds__(VNT) kw_residual(GroupArgs g) {
    __shared__ VS S;
    const int n = g.nx, m = g.nu, tid = threadIdx.x;
    const LeafItem it = sv::load_leaf(g.leaves, blockIdx.x);
    if (sv::skip_inst(g, it.inst)) return;
    const sv::Prob p = sv::load_prob(g.probs, it.inst);
    const sv::Prob c = sv::load_prob(g.corr ? g.corr : g.probs, it.inst);
    double rhs = 0.0, res = 0.0, obj = 0.0, zn = 0.0;
    const int len = uni(it.len);
    double *xs = S.x, *ws = S.wv, *ls = S.lamN;
    for (int s = 0; s < len; ++s) {
        const int64_t t = it.t0 + s;
        const double *x = p.x + t * n, *xn = x + n, *w = p.w + t * m;
        const double *lam = p.lam + t * n, *lamn = lam + n;
        const double *Qx = p.Qx + t * p.sQx, *Qw = p.Qw + t * p.sQw;
        const double *Qxw = p.Qxw ? p.Qxw + t * p.sQxw : nullptr;
        const double *A = p.A + t * p.sA, *B = p.B + t * p.sB;
        for (int i = tid; i < n; i += nthr()) {
            xs[i] = x[i];
            ls[i] = lamn[i];
            zn = fmax(zn, fmax(fabs(x[i]), fabs(lam[i])));
        }
        for (int i = tid; i < m; i += nthr()) {
            ws[i] = w[i];
            zn = fmax(zn, fabs(w[i]));
        }
        __syncthreads();
        // x row: Qx x + Qxw w - lam + A' lam+ ; lam+ row: A x + B w - x+ ;
        // w row: Qxw' x + Qw w + B' lam+.  A, B and Qxw are read once for
        // both of their products; Qx and Qw (symmetric) by columns.
        gemv<false>(Qx, n, xs, n, n, [&](int i, double v) { S.pt[i] = v; }, S.gred);
        gemv_both(A, n, ls, xs, n, n, [&](int i, double v) { S.av[i] = v; }, [&](int k, double v) { S.y[k] = v; },
                  S.gred);
        gemv_both(B, m, ls, ws, n, m, [&](int j, double v) { S.kk[j] = v; },
                  [&](int k, double v) { S.Psi[k] = v; }, S.gred);
        if (Qxw) {
            gemv_both(Qxw, m, xs, ws, n, m, [&](int j, double v) { S.gw[j] = v; },
                      [&](int k, double v) { S.d[k] = v; }, S.gred);
        } else {
            for (int i = tid; i < n; i += nthr()) S.d[i] = 0.0;
            for (int j = tid; j < m; j += nthr()) S.gw[j] = 0.0;
        }
        gemv<false>(Qw, m, ws, m, m, [&](int j, double v) { S.z[j] = v; }, S.gred);
        __syncthreads();
        double part = 0.0;
        for (int i = tid; i < n; i += nthr()) {
            const double lxi = p.lx ? p.lx[t * p.slx + i] : 0.0, ai = p.a ? p.a[t * p.sa + i] : 0.0;
            const double dlx = lxi + S.pt[i] + S.d[i] - lam[i] + S.av[i];
            const double da = ai + S.y[i] + S.Psi[i] - xn[i];
            if (g.corr) {
                const_cast<double *>(c.lx)[t * c.slx + i] = dlx;
                const_cast<double *>(c.a)[t * c.sa + i] = da;
            }
            rhs = fmax(rhs, fmax(fabs(lxi), fabs(ai)));
            res = fmax(res, fmax(fabs(dlx), fabs(da)));
            part += xs[i] * (0.5 * S.pt[i] + S.d[i] + lxi);
        }
        for (int j = tid; j < m; j += nthr()) {
            const double lwj = p.lw ? p.lw[t * p.slw + j] : 0.0;
            const double dlw = lwj + S.gw[j] + S.z[j] + S.kk[j];
            if (g.corr) const_cast<double *>(c.lw)[t * c.slw + j] = dlw;
            rhs = fmax(rhs, fabs(lwj));
            res = fmax(res, fabs(dlw));
            part += ws[j] * (0.5 * S.z[j] + lwj);
        }
        const double tot = block_sum(part, S);
        if (tid == 0) obj += tot + (p.c ? p.c[t * p.sc] : 0.0);
    }
    if (it.t0 == 0) {            // lam_0 row
        for (int i = tid; i < n; i += nthr()) {
            const double d0 = p.x[i] - p.x0[i];
            if (g.corr) const_cast<double *>(c.x0)[i] = d0;
            rhs = fmax(rhs, fabs(p.x0[i]));
            res = fmax(res, fabs(d0));
        }
    }
    if (it.flags & LEAF_LAST) {  // x_N row and the terminal cost
        const int64_t N = it.t0 + len;
        const double *x = p.x + N * n, *lam = p.lam + N * n;
        for (int i = tid; i < n; i += nthr()) xs[i] = x[i];
        __syncthreads();
        double part = 0.0;
        gemv<true>(p.QxN, n, xs, n, n, [&](int i, double qx) {
            const double lNi = p.lN ? p.lN[i] : 0.0;
            const double dN = lNi + qx - lam[i];
            if (g.corr) const_cast<double *>(c.lN)[i] = dN;
            zn = fmax(zn, fmax(fabs(x[i]), fabs(lam[i])));
            rhs = fmax(rhs, fabs(lNi));
            res = fmax(res, fabs(dN));
            part += x[i] * (0.5 * qx + lNi);
        }, S.gred);
        const double tot = block_sum(part, S);
        if (tid == 0) obj += tot + (p.cN ? p.cN[0] : 0.0);
    }
    rhs = sv::wave_max(rhs);
    res = sv::wave_max(res);
    zn = sv::wave_max(zn);
    __syncthreads();
    if (lane() == 0) {
        S.av[wave()] = rhs;
        S.pt[wave()] = res;
        S.y[wave()] = zn;
    }
    __syncthreads();
    if (tid == 0) {
        double *out = g.part + (int64_t)(g.leaf_base + blockIdx.x) * PART_N;
        double a = 0.0, b = 0.0, z = 0.0;
        for (int q = 0; q < nwav(); ++q) {
            a = fmax(a, S.av[q]);
            b = fmax(b, S.pt[q]);
            z = fmax(z, S.y[q]);
        }
        out[PART_RHS] = a;
        out[PART_RES] = b;
        out[PART_OBJ] = obj;
        out[PART_ZN] = z;
    }
}

// z += d over the leaf's stages (and x_N, lam_N for the last leaf); max |d|
// and max |z| per block (x, w, lam).
__global__ void __launch_bounds__(VNT) kw_update(GroupArgs g) {
    __shared__ double red[VNT / 64][6];
    const int n = g.nx, m = g.nu, tid = threadIdx.x;
    const LeafItem it = sv::load_leaf(g.leaves, blockIdx.x);
    if (sv::skip_inst(g, it.inst)) return;
    const sv::Prob p = sv::load_prob(g.probs, it.inst);
    const sv::Prob c = sv::load_prob(g.corr, it.inst);
    const int nst = uni(it.len) + ((it.flags & LEAF_LAST) ? 1 : 0);
    double mx[6] = {0, 0, 0, 0, 0, 0};
    {
        const int64_t b0 = (int64_t)it.t0 * n, cnt = (int64_t)nst * n;
        for (int64_t e = tid; e < cnt; e += nthr()) {
            const double dx = c.x[b0 + e], dl = c.lam[b0 + e];
            double xv = p.x[b0 + e], lv = p.lam[b0 + e];
            if (!g.measure_only) {
                xv += dx;
                lv += dl;
                p.x[b0 + e] = xv;
                p.lam[b0 + e] = lv;
            }
            mx[0] = fmax(mx[0], fabs(dx));
            mx[2] = fmax(mx[2], fabs(dl));
            mx[3] = fmax(mx[3], fabs(xv));
            mx[5] = fmax(mx[5], fabs(lv));
        }
    }
    {
        const int64_t b0 = (int64_t)it.t0 * m, cnt = (int64_t)it.len * m;
        for (int64_t e = tid; e < cnt; e += nthr()) {
            const double dw = c.w[b0 + e];
            double wv = p.w[b0 + e];
            if (!g.measure_only) {
                wv += dw;
                p.w[b0 + e] = wv;
            }
            mx[1] = fmax(mx[1], fabs(dw));
            mx[4] = fmax(mx[4], fabs(wv));
        }
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) mx[q] = sv::wave_max(mx[q]);
    if (lane() == 0)
        for (int q = 0; q < 6; ++q) red[wave()][q] = mx[q];
    __syncthreads();
    if (tid == 0) {
        double *out = g.part + (int64_t)(g.leaf_base + blockIdx.x) * PART_N;
        for (int q = 0; q < 6; ++q) {
            double v = 0.0;
            for (int w = 0; w < nwav(); ++w) v = fmax(v, red[w][q]);
            out[PART_DX + q] = v;
        }
    }
}

// ------------------------------------------------------------- launchers
// threads of a vector-line launch: all eight wavefronts for the larger
// shapes, four for n_x < 32, where each product is a few short rows and the
// extra waves cost more in synchronization than they bring in loads
int vthreads(const GroupArgs &g) { return g.nx >= 32 ? VNT : VNT / 2; }
int leaf_units(const GroupArgs &g) { return std::max(1, std::min<int>(g.nleaves, LB_LEAF_UNITS)); }

// the LDS-panel products serve the stages with n_x > 64
inline bool big_stage(const GroupArgs &g) { return g.nx > 64; }

template <class T, bool BF = false>
hipError_t launch_leaf_up(const GroupArgs &g, int, hipStream_t st) {
    if (big_stage(g))
        hipLaunchKernelGGL((kl_leaf_up<T, BF, true>), dim3(leaf_units(g)), dim3(LB_MT), 0, st, g);
    else
        hipLaunchKernelGGL((kl_leaf_up<T, BF, false>), dim3(leaf_units(g)), dim3(LB_MT), 0, st, g);
    return hipGetLastError();
}
hipError_t launch_tree(const GroupArgs &g, int grid, hipStream_t st) {
    if (big_stage(g))
        hipLaunchKernelGGL(kl_tree<true>, dim3(std::min(grid, LB_TREE_UNITS)), dim3(LB_MT), 0, st, g);
    else
        hipLaunchKernelGGL(kl_tree<false>, dim3(std::min(grid, LB_TREE_UNITS)), dim3(LB_MT), 0, st, g);
    return hipGetLastError();
}
template <class T, bool BF = false>
hipError_t launch_leaf_down(const GroupArgs &g, int, hipStream_t st) {
    if (g.ntop == 0) return hipSuccess;
    if (big_stage(g))
        hipLaunchKernelGGL((kl_leaf_down<T, BF, true>), dim3(leaf_units(g)), dim3(LB_MT), 0, st, g);
    else
        hipLaunchKernelGGL((kl_leaf_down<T, BF, false>), dim3(leaf_units(g)), dim3(LB_MT), 0, st, g);
    return hipGetLastError();
}
template <class TR>
hipError_t launch_vup(const GroupArgs &g, int, hipStream_t st) {
    hipLaunchKernelGGL((kw_leaf_up<TR>), dim3(g.nleaves), dim3(vthreads(g)), 0, st, g);
    return hipGetLastError();
}
hipError_t launch_vtree(const GroupArgs &g, int grid, hipStream_t st) {
    hipLaunchKernelGGL(kw_tree, dim3(grid), dim3(vthreads(g)), 0, st, g);
    return hipGetLastError();
}
template <class TR>
hipError_t launch_vdown(const GroupArgs &g, int, hipStream_t st) {
    hipLaunchKernelGGL((kw_leaf_down<TR>), dim3(g.nleaves), dim3(vthreads(g)), 0, st, g);
    return hipGetLastError();
}
hipError_t launch_residual(const GroupArgs &g, int grid, hipStream_t st) {
    hipLaunchKernelGGL(kw_residual, dim3(grid), dim3(vthreads(g)), 0, st, g);
    return hipGetLastError();
}
hipError_t launch_update(const GroupArgs &g, int grid, hipStream_t st) {
    hipLaunchKernelGGL(kw_update, dim3(grid), dim3(vthreads(g)), 0, st, g);
    return hipGetLastError();
}

}  // namespace lb

bool large_shape(int nx, int nu) { return nx >= 1 && nu >= 1 && nx <= lb::VMAX && nu <= lb::VMAX; }

Launcher large_factor(int which, bool fp32, bool bf16) {
    if (which == 1) return &lb::launch_tree;
    if (bf16) return which == 0 ? &lb::launch_leaf_up<float, true> : &lb::launch_leaf_down<float, true>;
    if (which == 0) return fp32 ? &lb::launch_leaf_up<float> : &lb::launch_leaf_up<double>;
    return fp32 ? &lb::launch_leaf_down<float> : &lb::launch_leaf_down<double>;
}

Launcher large_vector(int which, bool fp32) {
    if (which == 0) return fp32 ? &lb::launch_vup<float> : &lb::launch_vup<double>;
    if (which == 1) return &lb::launch_vtree;
    return fp32 ? &lb::launch_vdown<float> : &lb::launch_vdown<double>;
}

Launcher large_refine(int which) { return which == 0 ? &lb::launch_residual : &lb::launch_update; }

}  // namespace rs
