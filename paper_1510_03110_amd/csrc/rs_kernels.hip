// Kernels of the parallel Riccati Newton-step solve (fused factor + solve).
//
//   k_init       clears per-instance status words and the tree work queues
//   k_leaf_up    one workgroup per leaf: Alg. 4 on the leaf (or, for the
//                last leaf, elimination with the true terminal, Sec. 4.2);
//                writes the leaf's M1 message into its level-1 slot (Alg. 5)
//   k_tree       persistent work-queue kernel over the master levels: reduce
//                each master subproblem (Alg. 5, k >= 1), solve the top
//                problem (Alg. 6, k = m) and propagate the solution down to
//                level 1 (Alg. 6, k >= 1).  Items are queued so that every
//                item depends only on items queued before it; a workgroup
//                that takes an item waits on the completion flags of its
//                dependencies, which belong to workgroups that are already
//                running, so the wait always ends.
//   k_leaf_down  one workgroup per leaf: Alg. 1-3 on the leaf with the
//                parent's P, Psi, cbar and x (Alg. 6, k = 0); writes x, w, lam.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "rs_device.hpp"
#include "rs_launch.hpp"

namespace rs {

constexpr int SPIN_LIMIT = 1 << 26;   // bounded dependency wait (tens of seconds)

__global__ void k_init(int32_t *info, int count, int32_t *queues, int nq) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        info[2 * i] = 0;
        info[2 * i + 1] = -1;
    }
    if (i < nq) queues[i] = 0;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Work-table entries read into wave-uniform registers.
__device__ __forceinline__ LeafItem load_leaf(const LeafItem *tab, int i) {
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

template <class T, int NX, int NU>
struct LeafSmem {
    static constexpr size_t bytes =
        sizeof(Smem<T, NX, NU, true>) > sizeof(Smem<T, NX, NU, false>) ? sizeof(Smem<T, NX, NU, true>)
                                                                         : sizeof(Smem<T, NX, NU, false>);
};

// Scratch of the leaf solve, per stage: K (NU*NX) | k (NU) | P (NX*NX) | Psi (NX)
template <int NX, int NU>
struct LeafScratch {
    static constexpr int K = 0, k = NU * NX, P = NU * NX + NU, Psi = NU * NX + NU + NX * NX,
                         per_stage = NU * NX + NU + NX * NX + NX;
};

// ------------------------------------------------------------------ leaves
template <class T, int NX, int NU>
__global__ void __launch_bounds__(NT) k_leaf_up(GroupArgs g) {
    __shared__ __attribute__((aligned(16))) char raw[LeafSmem<T, NX, NU>::bytes];
    const LeafItem it = load_leaf(g.leaves, blockIdx.x);
    if ((it.flags & LEAF_TOP) || inst_skipped(g.probs, it.inst)) return;
    const DevProb p = load_prob(g.probs, it.inst);
    const SlotLayout SL{NX};
    double *out = g.slots + (int64_t)it.slot * SL.size();
    auto get = [&](int s) { return prob_stage(p, it.t0 + s); };
    if (!(it.flags & LEAF_LAST)) {
        auto &S = *reinterpret_cast<Smem<T, NX, NU, true> *>(raw);
        reduce_pass<T, NX, NU>(S, get, it.len, out, g.info, it.inst, it.t0, g.ident != nullptr);
    } else {
        auto &S = *reinterpret_cast<Smem<T, NX, NU, false> *>(raw);
        const int tid = threadIdx.x;
        for (int e = tid; e < NX * NX; e += NT) S.P[e] = (T)p.QxN[e];
        for (int i = tid; i < NX; i += NT) S.Psi[i] = p.lN ? -(T)p.lN[i] : T(0);
        if (tid == 0) S.cbar = p.cN ? (T)p.cN[0] : T(0);
        backward_pass<false, T, NX, NU>(
            S, get, it.len, g.info, it.inst, it.t0, 2, [](int, auto &) {}, [](int, auto &) {});
        for (int e = tid; e < NX * NX; e += NT) out[SL.Qx() + e] = (double)S.P[e];
        for (int i = tid; i < NX; i += NT) out[SL.lx() + i] = -(double)S.Psi[i];
        if (tid == 0) out[SL.c()] = (double)S.cbar;
    }
}

template <class T, int NX, int NU>
__global__ void __launch_bounds__(NT) k_leaf_down(GroupArgs g) {
    __shared__ __attribute__((aligned(16))) char raw[sizeof(Smem<T, NX, NU, false>)];
    auto &S = *reinterpret_cast<Smem<T, NX, NU, false> *>(raw);
    using SC = LeafScratch<NX, NU>;
    const LeafItem it = load_leaf(g.leaves, blockIdx.x);
    if (inst_skipped(g.probs, it.inst)) return;
    const DevProb p = load_prob(g.probs, it.inst);
    const SlotLayout SL{NX};
    const int tid = threadIdx.x;
    const bool known_end = (it.flags & (LEAF_LAST | LEAF_TOP)) != 0;
    const double *msg = (it.flags & LEAF_TOP) ? nullptr : g.slots + (int64_t)it.slot * SL.size();
    T *scr = reinterpret_cast<T *>(g.leaf_scratch) + it.scratch;
    // terminal cost to go of the leaf and its initial state (Alg. 6 messages)
    for (int e = tid; e < NX * NX; e += NT) S.P[e] = known_end ? (T)p.QxN[e] : (T)msg[SL.P() + e];
    for (int i = tid; i < NX; i += NT) {
        S.Psi[i] = known_end ? (p.lN ? -(T)p.lN[i] : T(0)) : (T)msg[SL.Psi() + i];
        S.x[i] = msg ? (T)msg[SL.xh() + i] : (T)p.x0[i];
    }
    if (tid == 0) S.cbar = known_end ? (p.cN ? (T)p.cN[0] : T(0)) : (T)msg[SL.cb()];
    auto get = [&](int s) { return prob_stage(p, it.t0 + s); };
    backward_pass<true, T, NX, NU>(
        S, get, it.len, g.info, it.inst, it.t0, 2, [](int, auto &) {},
        [&](int s, auto &Sm) {
            T *d = scr + (int64_t)s * SC::per_stage;
            for (int e = tid; e < NU * NX; e += NT) d[SC::K + e] = Sm.K[e];
            for (int e = tid; e < NX * NX; e += NT) d[SC::P + e] = Sm.P[e];
            for (int i = tid; i < NX; i += NT) d[SC::Psi + i] = Sm.Psi[i];
            for (int r = tid; r < NU; r += NT) d[SC::k + r] = Sm.kk[r];
        });
    if ((it.flags & LEAF_TOP) && p.obj) {
        // optimal value: cost to go at t = 0, 1/2 x0'P_0 x0 - Psi_0'x0 + cbar_0
        T part = 0;
        for (int i = tid; i < NX; i += NT) {
            T acc = 0;
            for (int k = 0; k < NX; ++k) acc += S.P[i * NX + k] * S.x[k];
            part += S.x[i] * (T(0.5) * acc - S.Psi[i]);
        }
        const T tot = block_sum(part, S);
        if (tid == 0) p.obj[0] = (double)(tot + S.cbar);
    }
    __syncthreads();
    forward_pass<T, NX, NU>(
        S, get, it.len,
        [&](int s, auto &Sm) {
            const T *d = scr + (int64_t)s * SC::per_stage;
            for (int e = tid; e < NU * NX; e += NT) Sm.K[e] = d[SC::K + e];
            for (int e = tid; e < NX * NX; e += NT) Sm.P[e] = d[SC::P + e];
            for (int i = tid; i < NX; i += NT) Sm.Psi[i] = d[SC::Psi + i];
            for (int r = tid; r < NU; r += NT) Sm.kk[r] = d[SC::k + r];
        },
        [&](int s, auto &Sm) {
            const int t = it.t0 + s;
            for (int i = tid; i < NX; i += NT) {
                T acc = -Sm.Psi[i];
                for (int k = 0; k < NX; ++k) acc += Sm.P[i * NX + k] * Sm.x[k];
                p.lam[(int64_t)t * NX + i] = (double)acc;      // lam_t = P_t x_t - Psi_t
                p.x[(int64_t)t * NX + i] = (double)Sm.x[i];
            }
            for (int r = tid; r < NU; r += NT) p.w[(int64_t)t * NU + r] = (double)Sm.wv[r];
        });
    if (known_end) {
        const int t = it.t0 + it.len;   // = N
        for (int i = tid; i < NX; i += NT) {
            T acc = p.lN ? (T)p.lN[i] : T(0);
            for (int k = 0; k < NX; ++k) acc += (T)p.QxN[i * NX + k] * S.x[k];
            p.lam[(int64_t)t * NX + i] = (double)acc;           // lam_N = QxN x_N + lN
            p.x[(int64_t)t * NX + i] = (double)S.x[i];
        }
    }
}

// -------------------------------------------------------------- the tree
template <int NX>
__device__ void tree_solve_item(Smem<double, NX, NX, false> &S, const TreeItem &it, const DevProb &p,
                                GroupArgs &g) {
    const SlotLayout SL{NX};
    const int tid = threadIdx.x;
    double *slots = g.slots;
    auto slot = [&](int s) { return slots + (int64_t)s * SL.size(); };
    const bool top = it.kind == ITEM_TOP;
    const double *msg = top ? nullptr : slot(it.out_slot);   // parent's M2 for this node
    const double *term = it.last ? slot(it.term_slot) : nullptr;
    for (int e = tid; e < NX * NX; e += NT) S.P[e] = term ? term[SL.Qx() + e] : msg[SL.P() + e];
    for (int i = tid; i < NX; i += NT) {
        S.Psi[i] = term ? -term[SL.lx() + i] : msg[SL.Psi() + i];
        S.x[i] = top ? p.x0[i] : msg[SL.xh() + i];
    }
    if (tid == 0) S.cbar = term ? term[SL.c()] : msg[SL.cb()];
    auto get = [&](int s) { return slot_stage(slot(it.first + s), NX, g.ident); };
    backward_pass<true, double, NX, NX>(
        S, get, it.count, g.info, it.inst, -1, 3,
        [&](int s, auto &Sm) {          // M2 for child s: cost to go at the end of stage s
            double *d = slot(it.first + s);
            for (int e = tid; e < NX * NX; e += NT) d[SL.P() + e] = Sm.P[e];
            for (int i = tid; i < NX; i += NT) d[SL.Psi() + i] = Sm.Psi[i];
            if (tid == 0) d[SL.cb()] = Sm.cbar;
        },
        [&](int s, auto &Sm) {          // master feedback of stage s for the forward pass
            double *d = slot(it.first + s);
            for (int e = tid; e < NX * NX; e += NT) d[SL.K() + e] = Sm.K[e];
            for (int i = tid; i < NX; i += NT) d[SL.k() + i] = Sm.kk[i];
        });
    if (top && p.obj) {
        double part = 0;
        for (int i = tid; i < NX; i += NT) {
            double acc = 0;
            for (int k = 0; k < NX; ++k) acc += S.P[i * NX + k] * S.x[k];
            part += S.x[i] * (0.5 * acc - S.Psi[i]);
        }
        const double tot = block_sum(part, S);
        if (tid == 0) p.obj[0] = tot + S.cbar;
    }
    __syncthreads();
    forward_pass<double, NX, NX>(
        S, get, it.count,
        [&](int s, auto &Sm) {
            const double *d = slot(it.first + s);
            for (int e = tid; e < NX * NX; e += NT) Sm.K[e] = d[SL.K() + e];
            for (int i = tid; i < NX; i += NT) Sm.kk[i] = d[SL.k() + i];
        },
        [&](int s, auto &Sm) {          // M2 for child s: its initial state
            double *d = slot(it.first + s);
            for (int i = tid; i < NX; i += NT) d[SL.xh() + i] = Sm.x[i];
        });
    if (it.last) {
        double *d = slot(it.term_slot);
        for (int i = tid; i < NX; i += NT) d[SL.xh() + i] = S.x[i];
    }
}

template <int NX>
__global__ void __launch_bounds__(NT) k_tree(GroupArgs g) {
    constexpr size_t B1 = sizeof(Smem<double, NX, NX, true>), B2 = sizeof(Smem<double, NX, NX, false>);
    __shared__ __attribute__((aligned(16))) char raw[B1 > B2 ? B1 : B2];
    __shared__ int s_item;
    const int tid = threadIdx.x;
    const SlotLayout SL{NX};
    for (;;) {
        if (tid == 0) s_item = atomicAdd(g.queue, 1);
        __syncthreads();
        const int idx = uni(s_item);
        __syncthreads();
        if (idx >= g.nitems) break;
        const TreeItem it = load_item(g.items, idx);
        if (tid == 0) {
            for (int d = 0; d < it.dep_count; ++d) {
                int spins = 0;
                while (__hip_atomic_load(&g.flags[it.dep_first + d], __ATOMIC_ACQUIRE,
                                         __HIP_MEMORY_SCOPE_AGENT) != g.epoch) {
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
            auto &S = *reinterpret_cast<Smem<double, NX, NX, true> *>(raw);
            reduce_pass<double, NX, NX>(S, get, it.count, slot(it.out_slot), g.info, it.inst, -1, g.ident != nullptr);
        } else if (it.kind == ITEM_UP_LAST) {
            auto &S = *reinterpret_cast<Smem<double, NX, NX, false> *>(raw);
            const double *term = slot(it.term_slot);
            for (int e = tid; e < NX * NX; e += NT) S.P[e] = term[SL.Qx() + e];
            for (int i = tid; i < NX; i += NT) S.Psi[i] = -term[SL.lx() + i];
            if (tid == 0) S.cbar = term[SL.c()];
            backward_pass<false, double, NX, NX>(
                S, get, it.count, g.info, it.inst, -1, 3, [](int, auto &) {}, [](int, auto &) {});
            double *out = slot(it.out_slot);
            for (int e = tid; e < NX * NX; e += NT) out[SL.Qx() + e] = S.P[e];
            for (int i = tid; i < NX; i += NT) out[SL.lx() + i] = -S.Psi[i];
            if (tid == 0) out[SL.c()] = S.cbar;
        } else {
            auto &S = *reinterpret_cast<Smem<double, NX, NX, false> *>(raw);
            tree_solve_item<NX>(S, it, p, g);
        }
        __threadfence();
        __syncthreads();
        if (tid == 0)
            __hip_atomic_store(&g.flags[idx], g.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        // keep the flag store and the next dequeue (both thread 0 only) in
        // separate regions: the loop's back edge must be taken by all lanes
        __syncthreads();
    }
}

// ---------------------------------------------------------------- launchers
template <class T, int NX, int NU>
static hipError_t launch_leaf_up(const GroupArgs &g, int, hipStream_t st) {
    hipLaunchKernelGGL((k_leaf_up<T, NX, NU>), dim3(g.nleaves), dim3(NT), 0, st, g);
    return hipGetLastError();
}
template <int NX>
static hipError_t launch_tree(const GroupArgs &g, int grid, hipStream_t st) {
    hipLaunchKernelGGL((k_tree<NX>), dim3(grid), dim3(NT), 0, st, g);
    return hipGetLastError();
}
template <class T, int NX, int NU>
static hipError_t launch_leaf_down(const GroupArgs &g, int, hipStream_t st) {
    hipLaunchKernelGGL((k_leaf_down<T, NX, NU>), dim3(g.nleaves), dim3(NT), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_init(int32_t *info, int count, int32_t *queues, int nq, hipStream_t st) {
    const int n = count > nq ? count : nq;
    hipLaunchKernelGGL(k_init, dim3((n + 255) / 256), dim3(256), 0, st, info, count, queues, nq);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// Shapes with generic (VALU) kernels; shapes whose dimensions are multiples
// of 16 use the matrix-core kernels instead (rs_kernels_mfma.hip), and the
// master levels use them whenever n_x is a multiple of 16.
#define RS_GENERIC_SHAPES(X) \
    X(1, 1) X(2, 1) X(2, 2) X(3, 2) X(4, 2) X(4, 4) X(6, 3) X(8, 4) X(16, 8) X(20, 10)

Launcher mfma_leaf_up(int nx, int nu);
Launcher mfma_leaf_down(int nx, int nu);
Launcher mfma_tree(int nx);

namespace {
struct GenericEntry {
    int nx, nu;
    Launcher up, tree, down;
};
const GenericEntry generic_table[] = {
#define RS_ENTRY(a, b) {a, b, &launch_leaf_up<double, a, b>, &launch_tree<a>, &launch_leaf_down<double, a, b>},
    RS_GENERIC_SHAPES(RS_ENTRY)
#undef RS_ENTRY
};
}  // namespace

const ShapeEntry *find_shape(int nx, int nu) {
    static ShapeEntry table[64];
    static int n = 0;
    static bool init = false;
    if (!init) {
        auto add = [&](int a, int b, Launcher up, Launcher tr, Launcher dn) {
            ShapeEntry e;
            e.nx = a;
            e.nu = b;
            e.large = false;
            e.lb = false;
            e.fp64[0] = mfma_leaf_up(a, b) ? mfma_leaf_up(a, b) : up;
            // the matrix-core tree sends its children their terminal costate,
            // which only the matrix-core leaf solve reads
            e.fp64[1] = (mfma_leaf_down(a, b) && mfma_tree(a)) ? mfma_tree(a) : tr;
            e.fp64[2] = mfma_leaf_down(a, b) ? mfma_leaf_down(a, b) : dn;
            for (int f = 0; f < 2; ++f)
                for (int k = 0; k < 3; ++k) {
                    e.factor[f][k] = mfma_factor(a, b, k, f == 1);
                    e.vsolve[f][k] = vector_solve(a, b, k, f == 1);
                }
            for (int k = 0; k < 3; ++k) e.factor[2][k] = nullptr;
            e.refine[0] = refine_kernel(a, b, 0);
            e.refine[1] = refine_kernel(a, b, 1);
            // no matrix-core form of the stored factorization: the large-block
            // kernels serve it (and mixed precision)
            e.lb = !e.factor[0][0] && large_shape(a, b);
            if (e.lb) {
                for (int f = 0; f < 2; ++f)
                    for (int k = 0; k < 3; ++k) {
                        e.factor[f][k] = large_factor(k, f == 1);
                        e.vsolve[f][k] = large_vector(k, f == 1);
                    }
                for (int k = 0; k < 3; ++k) e.factor[2][k] = large_factor(k, true, true);
                e.refine[0] = large_refine(0);
                e.refine[1] = large_refine(1);
            }
            e.scratch_per_stage = mfma_leaf_down(a, b) ? scratch_per_stage_fwd(a, b) : scratch_per_stage(a, b);
            if (e.fp64[0] && e.fp64[1] && e.fp64[2]) table[n++] = e;
        };
        for (const auto &g : generic_table) add(g.nx, g.nu, g.up, g.tree, g.down);
        const int mshapes[][2] = {{16, 16}, {32, 16}, {32, 32}};
        for (const auto &m : mshapes) add(m[0], m[1], nullptr, nullptr, nullptr);
        init = true;
    }
    for (int i = 0; i < n; ++i)
        if (table[i].nx == nx && table[i].nu == nu) return &table[i];
    // large-block family: any other shape up to 128 (entries made on first use)
    if (!large_shape(nx, nu)) return nullptr;
    static std::mutex mu;
    static std::map<std::pair<int, int>, ShapeEntry> large;
    std::lock_guard<std::mutex> lock(mu);
    auto it = large.find({nx, nu});
    if (it != large.end()) return &it->second;
    ShapeEntry e;
    e.nx = nx;
    e.nu = nu;
    e.large = true;
    e.lb = true;
    for (int k = 0; k < 3; ++k) {
        e.fp64[k] = nullptr;
        for (int f = 0; f < 2; ++f) {
            e.factor[f][k] = large_factor(k, f == 1);
            e.vsolve[f][k] = large_vector(k, f == 1);
        }
        e.factor[2][k] = large_factor(k, true, true);
    }
    e.refine[0] = large_refine(0);
    e.refine[1] = large_refine(1);
    if (mfma_factor_leaf32(nx, nu, 0)) {
        e.factor[1][0] = mfma_factor_leaf32(nx, nu, 0);
        e.factor[1][2] = mfma_factor_leaf32(nx, nu, 2);
    }
    e.scratch_per_stage = 1;      // leaf stage index = scratch offset
    return &large.emplace(std::make_pair(nx, nu), e).first->second;
}

}  // namespace rs
