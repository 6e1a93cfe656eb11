// C ABI of the parallel Riccati solver: argument checking, the tree plan
// (Alg. 5/6 levels and work lists), the workspace layout and the launches.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "rs.h"
#include "rs_launch.hpp"

using namespace rs;

namespace {

constexpr size_t ALIGN = 256;
// Instances with n_x = 16 or 32 and n_u below this are solved with their
// inputs padded to it (the matrix-core kernels' tile), see rs_pad.hip.
constexpr int PAD_NU = 16;
constexpr int RING = 4;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Group {
    int nx, nu;
    const ShapeEntry *shape;
    std::vector<int32_t> insts;
    std::vector<LeafItem> leaves;
    std::vector<TreeItem> items;
    int64_t nslots = 0;
    int64_t scratch_elems = 0;
    int max_depth = 0;
    int64_t leaf_stages = 0;
    int32_t leaf_base = 0;                  // global index of the group's first leaf
    int32_t ntop = 0;                       // single-leaf instances
    size_t off_leaves = 0, off_items = 0, off_flags = 0, off_slots = 0, off_scratch = 0, off_fstore = 0,
           off_fvec = 0;
    size_t off_lbw = 0, lbw_unit = 0;       // large-block workspace (per workgroup)
    int64_t ring_stages = 0;                // receding-horizon plans: record stages of the group
    int ring_m1 = 0;                        // and M1 cache blocks (3 n^2 doubles each)
    size_t off_m1 = 0;
    size_t off_ident = 0;                   // rank-revealing plans: n_x x n_x identity (in the tables)
    // receding-horizon plans: table and slot counts reserved for any window
    // position, so that the workspace size does not depend on it
    int64_t res_leaves = 0, res_items = 0, res_slots = 0;
};

}  // namespace

struct rs_plan_s {
    int32_t count = 0;
    int Ns = 16, branch = 4, top_max = 4, prec = RS_FP64, max_refine = 5;
    bool factored = false;          // workspace holds the stored factorization
    bool mixed = false;             // FP32 leaf factorization + FP64 refinement
    bool bf16 = false;              // ... with BF16 matrix-core products in the leaf stages
    bool via_factor = false;        // FP64 solve = stored factorization + solve (large-block shapes)
    bool receding = false;          // receding-horizon layout (rs_plan_create_ring)
    bool rank_reveal = false;       // rank-revealing master stages (RS_PLAN_RANK_REVEAL)
    bool report = false;            // per-instance report: K norm, FP64 residual, error estimate
    bool refine_ws = false;         // workspace holds the refinement tables (mixed or report)
    int32_t leaf_chunk = 0;         // > 0: leaves processed in chunks of this many (bounded factor store)
    bool check_inputs = false;      // RS_PLAN_CHECK_INPUTS: finite-input scan after every call
    bool superpose = true;          // stored factorization: superposition down pass (else RS_PLAN_REFACTOR_DOWN)
    size_t off_scan = 0;            // its per-instance first offending place
    rs_options opt{};               // options the plan was made with
    bool tables_dirty = false;      // host tables changed since the last upload
    hipEvent_t tables_ev = nullptr; // completion of the last table upload
    std::vector<int64_t> inst_start, inst_lo, inst_hi;
    int32_t total_leaves = 0;
    std::vector<InstInfo> inst;     // per instance: leaf range (refinement reductions)
    std::vector<size_t> off_cbuf;   // per instance: correction buffers (mixed)
    size_t off_inst = 0, off_conv = 0, off_stats = 0, off_part = 0;
    double tol = 1e-10;
    std::vector<int32_t> dims;          // (nx, nu, N) per instance
    std::vector<int32_t> inst_Ns, inst_branch;   // leaf length and branch per instance
    // rs_plan_create_split: leaf lengths and per-level master group sizes per
    // instance (empty: uniform Ns and branch)
    std::vector<std::vector<int32_t>> inst_lens, inst_brs;
    // input padding: per instance the caller's n_u (0: not padded; the plan
    // then uses n_u = PAD_NU) and the workspace offset of its padded arrays
    std::vector<int32_t> nu_user;
    std::vector<size_t> off_pad;
    std::vector<int32_t> pad_inst;      // padded instances in order
    size_t off_padargs = 0;
    std::vector<Group> groups;
    size_t off_probs = 0, off_info = 0, off_queues = 0, off_tables = 0, tables_bytes = 0;
    size_t total = 0;
    std::vector<char> tables;           // host image of every group's leaf and tree tables
    void *pinned_tables = nullptr;
    void *pinned_probs[RING] = {};
    hipEvent_t ev[RING] = {};
    bool ev_used[RING] = {};
    int ring = 0;
    void *bound_work = nullptr;
    std::vector<DevProb> last_probs;
    std::vector<PadArgs> last_pads;
    std::vector<DevProb> dp_host;       // descriptor images built per call (sized at creation)
    std::vector<PadArgs> pads_host;
    bool probs_valid = false;
    int32_t epoch = 0;
    int64_t last_refine = 0;
    // optional per-kernel timing with HIP events on the call's stream
    bool timing = false;
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
};

namespace {

// Build the tree of one instance (Sec. 5, Alg. 5/6) into its group.
// Leaves: ceil(N/Ns) batches of Ns stages, the last one ragged and holding
// the terminal cost (Sec. 4.2).  Level k >= 1 has S_k master stages plus a
// terminal; while S_k exceeds the top size its stages are grouped b at a time
// into master subproblems, the last group taking the terminal.
// Receding-horizon plans: interior ring blocks per instance (a window of N
// stages has at most N / Ns interior leaves) and the stages of its records
// (ring, then first-leaf and last-leaf areas of 2 Ns stages each).
int ring_blocks(int N, int Ns) { return N / Ns + 1; }
int64_t ring_stages(int N, int Ns) { return ((int64_t)ring_blocks(N, Ns) + 4) * Ns; }

struct Tmp {
    TreeItem it;
    int phase, level, inst, node;
    int dep_level, dep_lo, dep_hi;   // UP/TOP: child nodes at dep_level; DOWN: parent node
    bool dep_top;
};

void build_tree(Group &g, int inst, int L0, int base1, int b, int top_max, std::vector<Tmp> &tmp,
                const std::vector<int32_t> *brs = nullptr);

// Leaves of the given lengths (in stage order, summing to N) and master
// levels whose group size is brs[level - 1] (the last entry for deeper
// levels; the top problem of a level takes up to that many stages).
void build_instance_split(Group &g, int inst, const std::vector<int32_t> &lens, const std::vector<int32_t> &brs,
                          std::vector<Tmp> &tmp) {
    const int L0 = (int)lens.size();
    const int sps = g.shape->scratch_per_stage;
    if (L0 == 1) {
        LeafItem lf{inst, 0, lens[0], LEAF_LAST | LEAF_TOP, -1, 0, g.scratch_elems};
        g.leaves.push_back(lf);
        g.scratch_elems += (int64_t)lens[0] * sps;
        return;
    }
    const int base1 = (int)g.nslots;
    g.nslots += L0;
    int t0 = 0;
    for (int i = 0; i < L0; ++i) {
        LeafItem lf{inst, t0, lens[i], i == L0 - 1 ? LEAF_LAST : 0, base1 + i, 0, g.scratch_elems};
        g.leaves.push_back(lf);
        g.scratch_elems += (int64_t)lens[i] * sps;
        t0 += lens[i];
    }
    build_tree(g, inst, L0, base1, 0, 0, tmp, &brs);
}

void build_instance(Group &g, int inst, int N, int Ns, int b, int top_max, std::vector<Tmp> &tmp) {
    const int L0 = (N + Ns - 1) / Ns;
    const int sps = g.shape->scratch_per_stage;
    if (L0 == 1) {
        LeafItem lf{inst, 0, N, LEAF_LAST | LEAF_TOP, -1, 0, g.scratch_elems};
        g.leaves.push_back(lf);
        g.scratch_elems += (int64_t)N * sps;
        return;
    }
    const int base1 = (int)g.nslots;
    g.nslots += L0;
    for (int i = 0; i < L0; ++i) {
        const int t0 = i * Ns, len = std::min(Ns, N - t0);
        LeafItem lf{inst, t0, len, i == L0 - 1 ? LEAF_LAST : 0, base1 + i, 0, g.scratch_elems};
        g.leaves.push_back(lf);
        g.scratch_elems += (int64_t)len * sps;
    }
    build_tree(g, inst, L0, base1, b, top_max, tmp);
}

// Receding-horizon layout of one instance whose window starts at absolute
// stage `start`: leaf boundaries sit at absolute multiples of Ns, so a shift
// of the window leaves the interior leaves unchanged.  The first leaf runs
// from the window start to the second boundary after it (to the first if the
// start is on a boundary), so that every leaf but the last has at least Ns
// stages (Ns nu >= nx); with rank-revealing master stages (merge_first
// false), where a leaf of any length is reduced, it ends at the first
// boundary, which halves its length on average.  The last leaf ends with the
// window.  Interior leaf a
// (stages [a Ns, (a+1) Ns)) keeps its stored factorization in ring block
// a mod ring_blocks; the first and last leaves use areas of their own.
// Interior leaves with a in [lo, hi) are marked LEAF_REUSE.
// Stage offsets are relative to the instance's record base `rbase` (stages);
// `mbase` is its first M1 cache block.
void build_instance_ring(Group &g, int inst, int N, int Ns, int b, int top_max, int64_t start, int64_t lo,
                         int64_t hi, int64_t rbase, int mbase, bool merge_first, std::vector<Tmp> &tmp) {
    const int sps = g.shape->scratch_per_stage;
    const int nblocks = ring_blocks(N, Ns);
    const int64_t first_end = (start / Ns + ((start % Ns == 0 || !merge_first) ? 1 : 2)) * (int64_t)Ns,
                  end = start + N;
    const int64_t edge_first = rbase + (int64_t)nblocks * Ns, edge_last = edge_first + 2 * (int64_t)Ns;
    if (end <= first_end) {
        LeafItem lf{inst, 0, N, LEAF_LAST | LEAF_TOP, -1, -1, edge_first * sps};
        g.leaves.push_back(lf);
        return;
    }
    const int64_t last_a = (end - 1) / Ns;          // block of the last stage
    const int L0 = 1 + (int)(last_a - first_end / Ns) + 1 - (last_a * Ns < first_end ? 1 : 0);
    const int base1 = (int)g.nslots;
    g.nslots += L0;
    int i = 0;
    g.leaves.push_back(LeafItem{inst, 0, (int)(first_end - start), L0 == 1 ? LEAF_LAST : 0, base1 + i++, -1,
                                edge_first * sps});
    for (int64_t a = first_end / Ns; a < last_a; ++a) {
        const int blk = (int)(a % nblocks);
        const int flags = (a >= lo && a < hi) ? LEAF_REUSE : 0;
        g.leaves.push_back(LeafItem{inst, (int)(a * Ns - start), Ns, flags, base1 + i++, mbase + blk,
                                    (rbase + (int64_t)blk * Ns) * sps});
    }
    if (last_a * Ns >= first_end)
        g.leaves.push_back(LeafItem{inst, (int)(last_a * Ns - start), (int)(end - last_a * Ns), LEAF_LAST, base1 + i++,
                                    -1, edge_last * sps});
    build_tree(g, inst, L0, base1, b, top_max, tmp);
}

void build_tree(Group &g, int inst, int L0, int base1, int b, int top_max, std::vector<Tmp> &tmp,
                const std::vector<int32_t> *brs) {
    // group size and largest top problem of a level (uniform unless brs)
    auto br = [&](int lev) { return brs ? (*brs)[std::min<size_t>((size_t)lev - 1, brs->size() - 1)] : b; };
    auto tmx = [&](int lev) { return brs ? br(lev) : top_max; };
    int level = 1, S = L0 - 1, lvl_base = base1, prev_nodes = L0;
    for (;;) {
        const int bl = br(level);
        if (S <= tmx(level)) {
            Tmp t{};
            t.it = TreeItem{ITEM_TOP, inst, level, lvl_base, S, 1, lvl_base + S, -1, 0, 0};
            t.phase = 0;
            t.level = level;
            t.inst = inst;
            t.node = 0;
            t.dep_level = level - 1;
            t.dep_lo = 0;
            t.dep_hi = level > 1 ? prev_nodes : 0;
            tmp.push_back(t);
            g.max_depth = std::max(g.max_depth, level);
            break;
        }
        const int Lk = (S + bl - 1) / bl;
        const int nb = (int)g.nslots;
        g.nslots += Lk;
        const int Lnext = Lk - 1;                 // stages at the next level
        const int bn = br(level + 1);
        const bool next_is_top = Lnext <= tmx(level + 1);
        const int Lnext_nodes = next_is_top ? 1 : (Lnext + bn - 1) / bn;
        for (int j = 0; j < Lk; ++j) {
            const int first = lvl_base + j * bl, count = std::min(bl, S - j * bl);
            const int last = (j == Lk - 1) ? 1 : 0;
            Tmp u{};
            u.it = TreeItem{last ? ITEM_UP_LAST : ITEM_UP, inst, level, first, count, last,
                            last ? lvl_base + S : -1, nb + j, 0, 0};
            u.phase = 0;
            u.level = level;
            u.inst = inst;
            u.node = j;
            u.dep_level = level - 1;
            u.dep_lo = j * bl;
            u.dep_hi = level > 1 ? j * bl + count + last : 0;
            tmp.push_back(u);
            Tmp d = u;
            d.it.kind = ITEM_DOWN;
            d.phase = 1;
            d.dep_level = level + 1;
            d.dep_top = next_is_top;
            d.dep_lo = next_is_top ? 0 : std::min(j / bn, Lnext_nodes - 1);
            d.dep_hi = d.dep_lo + 1;
            tmp.push_back(d);
        }
        S = Lnext;
        lvl_base = nb;
        prev_nodes = Lk;
        ++level;
    }
}

void finalize_items(Group &g, std::vector<Tmp> &tmp) {
    std::stable_sort(tmp.begin(), tmp.end(), [](const Tmp &a, const Tmp &b) {
        const int la = a.phase == 0 ? a.level : -a.level, lb = b.phase == 0 ? b.level : -b.level;
        return std::make_tuple(a.phase, la, a.inst, a.node) < std::make_tuple(b.phase, lb, b.inst, b.node);
    });
    // index of (phase, inst, level, node); TOP items are looked up as phase 0
    std::map<std::tuple<int, int, int, int>, int> where;
    for (size_t i = 0; i < tmp.size(); ++i)
        where[std::make_tuple(tmp[i].phase, tmp[i].inst, tmp[i].level, tmp[i].node)] = (int)i;
    g.items.resize(tmp.size());
    for (size_t i = 0; i < tmp.size(); ++i) {
        TreeItem it = tmp[i].it;
        const Tmp &t = tmp[i];
        if (t.phase == 0) {
            if (t.dep_hi > t.dep_lo) {
                it.dep_first = where.at(std::make_tuple(0, t.inst, t.dep_level, t.dep_lo));
                it.dep_count = t.dep_hi - t.dep_lo;
            } else {
                it.dep_first = 0;
                it.dep_count = 0;
            }
        } else {
            const int ph = t.dep_top ? 0 : 1;
            it.dep_first = where.at(std::make_tuple(ph, t.inst, t.dep_level, t.dep_lo));
            it.dep_count = 1;
        }
        g.items[i] = it;
    }
}

bool valid_ptr_set(const rs_problem &p) {
    return p.Qx && p.Qw && p.A && p.B && p.QxN && p.x0 && p.x && p.w && p.lam;
}

rs_status to_status(hipError_t e) { return e == hipSuccess ? RS_OK : RS_ERR_HIP; }

hipEvent_t take_event(rs_plan_s *P) {
    hipEvent_t e = nullptr;
    if (!P->pool.empty()) {
        e = P->pool.back();
        P->pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
    }
    return e;
}

// roctx range over a host-side span (a public call, or the launch of one
// kernel kind): a profiler with marker tracing (rocprofv3 --marker-trace)
// shows the calls and the kernel kinds they launch by name.
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

// Kernel kind names (the order of rs_plan_kernel_times).
const char *kind_name(int kind) {
    static const char *const names[KK_COUNT] = {
        "rs.init", "rs.leaf_up", "rs.tree", "rs.leaf_down", "rs.factor_leaf_up", "rs.factor_tree",
        "rs.factor_leaf_down", "rs.solve_leaf_up", "rs.solve_tree", "rs.solve_leaf_down", "rs.residual",
        "rs.update", "rs.check", "rs.report", "rs.kind14", "rs.kind15"};
    return kind >= 0 && kind < KK_COUNT ? names[kind] : "rs.kernel";
}

// Launch one kernel of the given kind, inside a roctx range of its kind and
// bracketed by timing events when the plan's timing mode is on.
template <class F>
hipError_t timed(rs_plan_s *P, int kind, hipStream_t st, F &&launch) {
    Range range(kind_name(kind));
    if (!P->timing) return launch();
    hipEvent_t a = take_event(P), b = take_event(P);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, st);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, st);
    P->recs.push_back({kind, a, b});
    return e;
}

// Pinned host staging for the uploads of plan tables and problem
// descriptors, and the events that guard its reuse.  Taken at plan creation
// where a device is present, so that no call on the plan allocates; without
// a device (host-only plan inspection) the first call takes it instead.
void alloc_staging(rs_plan_s *P) {
    const size_t pbytes = sizeof(DevProb) * P->dp_host.size() + sizeof(PadArgs) * P->pad_inst.size();
    if (P->tables_bytes && !P->pinned_tables) {
        if (hipHostMalloc(&P->pinned_tables, P->tables_bytes) != hipSuccess) {
            P->pinned_tables = nullptr;
            (void)hipGetLastError();
            return;
        }
        if (hipEventCreateWithFlags(&P->tables_ev, hipEventDisableTiming) != hipSuccess) {
            P->tables_ev = nullptr;
            (void)hipGetLastError();
            return;
        }
    }
    for (int r = 0; r < RING; ++r) {
        if (P->pinned_probs[r]) continue;
        if (hipHostMalloc(&P->pinned_probs[r], pbytes) != hipSuccess) {
            P->pinned_probs[r] = nullptr;
            (void)hipGetLastError();
            return;
        }
        if (hipEventCreateWithFlags(&P->ev[r], hipEventDisableTiming) != hipSuccess) {
            P->ev[r] = nullptr;
            (void)hipGetLastError();
            return;
        }
    }
}

bool staging_ready(const rs_plan_s *P) {
    if (P->tables_bytes && (!P->pinned_tables || !P->tables_ev)) return false;
    for (int r = 0; r < RING; ++r)
        if (!P->pinned_probs[r] || !P->ev[r]) return false;
    return true;
}

}  // namespace

extern "C" {

const char *rs_status_string(rs_status s) {
    switch (s) {
    case RS_OK: return "ok";
    case RS_ERR_ARG: return "invalid argument";
    case RS_ERR_NOT_SPD: return "G not positive definite";
    case RS_ERR_SINGULAR_MASTER: return "singular reduced master block";
    case RS_ERR_NOT_CONVERGED: return "refinement did not converge";
    case RS_ERR_NOMEM: return "workspace too small";
    case RS_ERR_HIP: return "HIP runtime error";
    case RS_ERR_UNSUPPORTED: return "unsupported shape or option";
    }
    return "unknown status";
}

static rs_status plan_create(int32_t count, const int32_t *dims_in, int stride, const rs_options *opt,
                             rs_plan *out, const int32_t *leaf_off = nullptr, const int32_t *leaf_len = nullptr,
                             const int32_t *branch_off = nullptr, const int32_t *branch = nullptr) {
    if (!out || !dims_in || count < 1) return RS_ERR_ARG;
    *out = nullptr;
    rs_plan_s *P = new (std::nothrow) rs_plan_s();
    if (!P) return RS_ERR_NOMEM;
    if (opt) {
        if (opt->Ns < 0 || opt->branch < 0 || opt->branch == 1 || opt->max_refine < 0 || opt->tol < 0 ||
            opt->leaf_chunk < 0) {
            delete P;
            return RS_ERR_ARG;
        }
        if (opt->precision != RS_FP64 && opt->precision != RS_MIXED_FP32 && opt->precision != RS_MIXED_BF16) {
            delete P;
            return RS_ERR_UNSUPPORTED;
        }
        P->prec = opt->precision;
        P->mixed = opt->precision == RS_MIXED_FP32 || opt->precision == RS_MIXED_BF16;
        P->bf16 = opt->precision == RS_MIXED_BF16;
        P->factored = P->mixed || (opt->flags & RS_PLAN_FACTORED) != 0;
        P->rank_reveal = (opt->flags & RS_PLAN_RANK_REVEAL) != 0;
        P->report = (opt->flags & RS_PLAN_REPORT) != 0;
        P->leaf_chunk = opt->leaf_chunk;
        P->check_inputs = (opt->flags & RS_PLAN_CHECK_INPUTS) != 0;
        P->superpose = (opt->flags & RS_PLAN_REFACTOR_DOWN) == 0;
        if (opt->Ns > 0) P->Ns = opt->Ns;
        if (opt->branch > 0) P->branch = opt->branch;
        P->max_refine = opt->max_refine > 0 ? opt->max_refine : (P->bf16 ? 20 : 5);
        if (opt->tol > 0) P->tol = opt->tol;
    }
    if (opt) P->opt = *opt;
    P->refine_ws = P->mixed || P->report;
    P->top_max = P->branch;
    P->count = count;
    P->dims.resize(3 * (size_t)count);
    P->inst_Ns.resize(count);
    P->inst_lens.resize(count);
    P->inst_brs.resize(count);
    P->nu_user.assign(count, 0);
    P->off_pad.assign(count, 0);
    P->inst_branch.resize(count);
    for (int i = 0; i < count; ++i) {
        for (int k = 0; k < 3; ++k) P->dims[3 * i + k] = dims_in[(size_t)stride * i + k];
        const int ns = stride >= 5 ? dims_in[(size_t)stride * i + 3] : 0;
        const int br = stride >= 5 ? dims_in[(size_t)stride * i + 4] : 0;
        if (ns < 0 || br < 0 || br == 1) {
            delete P;
            return RS_ERR_ARG;
        }
        P->inst_Ns[i] = ns > 0 ? ns : P->Ns;
        P->inst_branch[i] = br > 0 ? br : P->branch;
        if (stride >= 8) {
            const int32_t *d = dims_in + (size_t)stride * i;
            if (d[5] < 0) {
                delete P;
                return RS_ERR_ARG;
            }
            P->inst_start.push_back(d[5]);
            P->inst_lo.push_back(d[6]);
            P->inst_hi.push_back(d[7]);
        }
    }
    if (stride >= 8) {
        // records live at fixed places across calls: the solve always runs on
        // the stored factorization
        P->receding = true;
        P->factored = true;
        P->via_factor = !P->mixed;
    }
    const int32_t *dims = P->dims.data();
    std::map<std::pair<int, int>, int> gidx;
    std::vector<int> inst_group(count);
    for (int i = 0; i < count; ++i) {
        const int nx = dims[3 * i], nu = dims[3 * i + 1], N = dims[3 * i + 2];
        if (nx < 1 || nu < 1 || N < 1) {
            delete P;
            return RS_ERR_ARG;
        }
        // without the rank-revealing form a multi-leaf instance needs
        // Ns*nu >= nx or the reduced input weight Q_w_hat = S Qbar^{-1} S' is
        // singular (Sec. 4.2 remark)
        if (leaf_off) {
            const int nl = leaf_off[i + 1] - leaf_off[i], nbr = branch_off[i + 1] - branch_off[i];
            if (nl < 1 || nbr < 1) {
                delete P;
                return RS_ERR_ARG;
            }
            std::vector<int32_t> lens(leaf_len + leaf_off[i], leaf_len + leaf_off[i + 1]);
            std::vector<int32_t> brs(branch + branch_off[i], branch + branch_off[i + 1]);
            int64_t sum = 0;
            bool ok = true;
            for (int k = 0; k < nl; ++k) {
                ok = ok && lens[k] >= 1;
                sum += lens[k];
                if (!P->rank_reveal && nl > 1 && k < nl - 1 && (int64_t)lens[k] * nu < nx) ok = false;
            }
            for (int32_t v : brs) ok = ok && v >= 2;
            if (!ok || sum != N) {
                delete P;
                return RS_ERR_ARG;
            }
            P->inst_lens[i] = std::move(lens);
            P->inst_brs[i] = std::move(brs);
        } else if (!P->rank_reveal && N > P->inst_Ns[i] && (int64_t)P->inst_Ns[i] * nu < nx) {
            delete P;
            return RS_ERR_ARG;
        }
        // n_u below the matrix-core tile at n_x = 16 or 32: padded inputs
        // (not in receding-horizon plans, whose records are windows of
        // caller-owned rings, nor with BF16 products)
        int nuk = nu;
        if (nu < PAD_NU && (nx == 16 || nx == 32) && !P->receding && !P->bf16 &&
            !(P->opt.flags & RS_PLAN_NATIVE_TILES)) {
            P->nu_user[i] = nu;
            P->dims[3 * i + 1] = PAD_NU;
            P->pad_inst.push_back(i);
            nuk = PAD_NU;
        }
        const ShapeEntry *se = find_shape(nx, nuk);
        const int f32 = P->mixed ? 1 : 0, fac = P->bf16 ? 2 : f32;
        if (se && se->large && !P->mixed) {
            // no fused kernels: the FP64 solve runs on the stored factorization
            P->factored = true;
            P->via_factor = true;
        }
        if (!se || (P->factored && !(se->factor[fac][0] && se->vsolve[f32][0])) || (P->refine_ws && !se->refine[0])) {
            delete P;
            return RS_ERR_UNSUPPORTED;
        }
        auto key = std::make_pair(nx, nuk);
        if (!gidx.count(key)) {
            gidx[key] = (int)P->groups.size();
            Group g;
            g.nx = nx;
            g.nu = nuk;
            g.shape = se;
            P->groups.push_back(g);
        }
        inst_group[i] = gidx[key];
        P->groups[inst_group[i]].insts.push_back(i);
    }
    P->inst.assign(count, InstInfo{});
    for (auto &g : P->groups) {
        std::vector<Tmp> tmp;
        g.leaf_base = P->total_leaves;
        for (int inst : g.insts) {
            const int before = (int)g.leaves.size();
            if (P->receding) {
                const int N = dims[3 * inst + 2], Ns = P->inst_Ns[inst];
                build_instance_ring(g, inst, N, Ns, P->inst_branch[inst], P->inst_branch[inst], P->inst_start[inst],
                                    P->inst_lo[inst], P->inst_hi[inst], g.ring_stages, g.ring_m1, !P->rank_reveal,
                                    tmp);
                g.ring_stages += ring_stages(N, Ns);
                g.ring_m1 += ring_blocks(N, Ns);
                // a window has between N/Ns - 1 and N/Ns + 2 leaves
                int64_t mi = 0, ms = 0;
                for (int L = std::max(1, N / Ns - 2); L <= N / Ns + 2; ++L) {
                    if (L == 1) continue;
                    Group d;
                    d.shape = g.shape;
                    d.nslots = L;
                    std::vector<Tmp> t;
                    build_tree(d, 0, L, 0, P->inst_branch[inst], P->inst_branch[inst], t);
                    mi = std::max<int64_t>(mi, (int64_t)t.size());
                    ms = std::max<int64_t>(ms, d.nslots);
                }
                g.res_leaves += N / Ns + 2;
                g.res_items += mi;
                g.res_slots += ms;
            } else if (!P->inst_lens[inst].empty()) {
                build_instance_split(g, inst, P->inst_lens[inst], P->inst_brs[inst], tmp);
            } else {
                build_instance(g, inst, dims[3 * inst + 2], P->inst_Ns[inst], P->inst_branch[inst],
                               P->inst_branch[inst], tmp);
            }
            InstInfo &in = P->inst[inst];
            in.first_leaf = g.leaf_base + before;
            in.nleaves = (int)g.leaves.size() - before;
            in.nx = g.nx;
            in.nu = g.nu;
            in.N = dims[3 * inst + 2];
        }
        P->total_leaves += (int32_t)g.leaves.size();
        for (auto &lf : g.leaves) g.ntop += (lf.flags & LEAF_TOP) ? 1 : 0;
        finalize_items(g, tmp);
    }
    // leaf-chunked solves: FP64 large-block plans only (their solve is the
    // stored factorization followed by the solve on it, both per leaf)
    if (P->leaf_chunk > 0) {
        bool ok = !P->mixed && !P->receding && P->pad_inst.empty();
        for (auto &g : P->groups) ok = ok && g.shape->large && g.shape->lb;
        if (!ok) {
            delete P;
            return RS_ERR_UNSUPPORTED;
        }
    }
    // workspace layout
    size_t off = 0;
    P->off_probs = off;                 // user problems, then (mixed) the correction problems,
    P->off_padargs = off + sizeof(DevProb) * count * (P->refine_ws ? 2 : 1);   // then the padding jobs
    off = align_up(P->off_padargs + sizeof(PadArgs) * P->pad_inst.size());
    P->off_info = off;
    off = align_up(off + sizeof(int32_t) * 2 * count);
    if (P->check_inputs) {
        P->off_scan = off;
        off = align_up(off + sizeof(int32_t) * count);
    }
    P->off_queues = off;
    off = align_up(off + sizeof(int32_t) * P->groups.size());
    if (P->receding) {
        // the stored factorization first: its place depends only on the
        // instances' shapes, horizons and leaf lengths, not on the window
        // positions, so consecutive receding-horizon plans share it
        for (auto &g : P->groups) {
            const size_t rec = P->mixed ? sizeof(float) : sizeof(double);
            g.leaf_stages = g.ring_stages;
            g.off_fstore = off;
            off = align_up(off + rec * (size_t)g.leaf_stages * LeafRec{g.nx, g.nu}.per_stage());
            g.off_fvec = off;
            off = align_up(off + sizeof(double) * (size_t)g.leaf_stages * LeafRec{g.nx, g.nu}.vec());
            g.off_m1 = off;
            off = align_up(off + sizeof(double) * 3 * (size_t)g.nx * g.nx * (size_t)g.ring_m1);
        }
    }
    P->off_tables = off;
    for (auto &g : P->groups) {
        g.off_leaves = off;
        off = align_up(off + sizeof(LeafItem) * std::max<size_t>(g.leaves.size(), (size_t)g.res_leaves));
        g.off_items = off;
        off = align_up(off + sizeof(TreeItem) * std::max<size_t>(g.items.size(), (size_t)g.res_items));
        if (P->rank_reveal) {
            g.off_ident = off;
            off = align_up(off + sizeof(double) * (size_t)g.nx * g.nx);
        }
    }
    P->off_inst = off;
    off = align_up(off + sizeof(InstInfo) * count);
    P->tables_bytes = off - P->off_tables;
    for (auto &g : P->groups) {
        g.off_flags = off;
        off = align_up(off + sizeof(int32_t) * std::max<size_t>({(size_t)1, g.items.size(), (size_t)g.res_items}));
    }
    for (auto &g : P->groups) {
        g.off_slots = off;
        off = align_up(off + sizeof(double) * SlotLayout{g.nx}.size() * (size_t)std::max(g.nslots, g.res_slots));
        g.off_scratch = off;
        const size_t esz = sizeof(double);
        off = align_up(off + esz * (size_t)g.scratch_elems);
        if (!P->receding) g.leaf_stages = g.scratch_elems / g.shape->scratch_per_stage;
        if (g.shape->lb && P->factored) {
            const int64_t units =
                std::max<int64_t>(std::min<int64_t>(std::max<int64_t>((int64_t)g.leaves.size(), g.res_leaves), LB_LEAF_UNITS),
                                  std::min<int64_t>(std::max<int64_t>((int64_t)g.items.size(), g.res_items), LB_TREE_UNITS));
            g.lbw_unit = large_unit_bytes(g.nx, g.nu);
            g.off_lbw = off;
            off = align_up(off + g.lbw_unit * (size_t)std::max<int64_t>(units, 1));
        }
        if (P->receding) continue;
        g.off_fstore = off;
        if (P->factored) {
            // a leaf-chunked plan stores the records of one chunk of leaves
            int64_t stages = g.leaf_stages;
            if (P->leaf_chunk > 0) {
                stages = 0;
                for (size_t lo = 0; lo < g.leaves.size(); lo += (size_t)P->leaf_chunk) {
                    const size_t hi = std::min(g.leaves.size(), lo + (size_t)P->leaf_chunk);
                    int64_t cs = 0;
                    for (size_t k = lo; k < hi; ++k) cs += g.leaves[k].len;
                    stages = std::max(stages, cs);
                }
            }
            const size_t rec = P->mixed ? sizeof(float) : sizeof(double);
            off = align_up(off + rec * (size_t)stages * LeafRec{g.nx, g.nu}.per_stage());
            g.off_fvec = off;
            off = align_up(off + sizeof(double) * (size_t)stages * LeafRec{g.nx, g.nu}.vec());
        }
    }
    if (P->refine_ws) {
        P->off_conv = off;                 // conv[count] | active[max_refine + 1]
        off = align_up(off + sizeof(int32_t) * (count + P->max_refine + 1));
        P->off_stats = off;
        off = align_up(off + sizeof(double) * ST_N * count);
        P->off_part = off;
        int64_t res_total = 0;
        for (auto &g : P->groups) res_total += std::max<int64_t>((int64_t)g.leaves.size(), g.res_leaves);
        off = align_up(off + sizeof(double) * PART_N * (size_t)res_total);
        // per instance: xbar0' nx | a' N nx | lx' N nx | lw' N nu | lN' nx | dx (N+1) nx | dw N nu | dlam (N+1) nx
        P->off_cbuf.resize(count);
        for (int i = 0; i < count; ++i) {
            const size_t nx = dims[3 * i], nu = dims[3 * i + 1], N = dims[3 * i + 2];
            P->off_cbuf[i] = off;
            off = align_up(off + sizeof(double) * (nx + 2 * N * nx + N * nu + nx + 2 * (N + 1) * nx + N * nu));
        }
    }
    for (int i : P->pad_inst) {
        // B, Q_xw (N nx x PAD_NU), Q_w (N PAD_NU^2), l_w and w (N PAD_NU)
        const size_t nx = dims[3 * i], N = dims[3 * i + 2];
        P->off_pad[i] = off;
        off = align_up(off + sizeof(double) * N * (2 * nx * PAD_NU + PAD_NU * PAD_NU + 2 * PAD_NU));
    }
    P->total = off;
    P->tables.assign(P->tables_bytes, 0);
    std::memcpy(P->tables.data() + (P->off_inst - P->off_tables), P->inst.data(), sizeof(InstInfo) * count);
    for (auto &g : P->groups) {
        if (!g.leaves.empty())
            std::memcpy(P->tables.data() + (g.off_leaves - P->off_tables), g.leaves.data(),
                        sizeof(LeafItem) * g.leaves.size());
        if (!g.items.empty())
            std::memcpy(P->tables.data() + (g.off_items - P->off_tables), g.items.data(),
                        sizeof(TreeItem) * g.items.size());
        if (P->rank_reveal) {
            double *I = reinterpret_cast<double *>(P->tables.data() + (g.off_ident - P->off_tables));
            for (int i = 0; i < g.nx; ++i) I[(size_t)i * g.nx + i] = 1.0;
        }
    }
    const size_t nprob = (size_t)count * (P->refine_ws ? 2 : 1);
    P->dp_host.resize(nprob);
    P->last_probs.reserve(nprob);
    P->pads_host.reserve(P->pad_inst.size());
    P->last_pads.reserve(P->pad_inst.size());
    *out = P;
    return RS_OK;
}

// A plan handed to the caller takes its pinned staging now, so that no call
// on it allocates.  (The plans that rs_plan_ring_update builds only for their
// tables take none: pinned allocation and release synchronize the device,
// which would serialize every serving launch.)
static rs_status with_staging(rs_status s, rs_plan *out) {
    if (s == RS_OK) alloc_staging(*out);
    return s;
}

rs_status rs_plan_create(int32_t count, const int32_t *dims, const rs_options *opt, rs_plan *out) {
    return with_staging(plan_create(count, dims, 3, opt, out), out);
}

rs_status rs_plan_create_ex(int32_t count, const int32_t *dims5, const rs_options *opt, rs_plan *out) {
    return with_staging(plan_create(count, dims5, 5, opt, out), out);
}

rs_status rs_plan_create_ring(int32_t count, const int32_t *dims8, const rs_options *opt, rs_plan *out) {
    return with_staging(plan_create(count, dims8, 8, opt, out), out);
}

rs_status rs_plan_create_split(int32_t count, const int32_t *dims, const int32_t *leaf_off, const int32_t *leaf_len,
                               const int32_t *branch_off, const int32_t *branch, const rs_options *opt, rs_plan *out) {
    if (!leaf_off || !leaf_len || !branch_off || !branch) return RS_ERR_ARG;
    return with_staging(plan_create(count, dims, 3, opt, out, leaf_off, leaf_len, branch_off, branch), out);
}

rs_status rs_plan_ring_update(rs_plan P, const int32_t *dims8) {
    if (!P || !P->receding || !dims8) return RS_ERR_ARG;
    rs_plan Q = nullptr;
    rs_status s = plan_create(P->count, dims8, 8, &P->opt, &Q);
    if (s != RS_OK) return s;
    // the instance list and every workspace offset must be unchanged
    bool same = Q->total == P->total && Q->dims == P->dims && Q->groups.size() == P->groups.size() &&
                Q->off_tables == P->off_tables && Q->tables_bytes == P->tables_bytes;
    for (size_t i = 0; same && i < P->groups.size(); ++i) {
        const Group &a = P->groups[i], &b = Q->groups[i];
        same = a.nx == b.nx && a.nu == b.nu && a.off_fstore == b.off_fstore && a.off_m1 == b.off_m1 &&
               a.off_slots == b.off_slots && a.off_flags == b.off_flags && a.off_lbw == b.off_lbw &&
               a.insts == b.insts;
    }
    if (!same) {
        rs_plan_destroy(Q);
        return RS_ERR_ARG;
    }
    // new leaves, tree items and instance tables; pinned buffers, events and
    // the bound workspace (with its stored factorization) stay
    std::swap(P->groups, Q->groups);
    std::swap(P->inst, Q->inst);
    std::swap(P->tables, Q->tables);
    std::swap(P->inst_start, Q->inst_start);
    std::swap(P->inst_lo, Q->inst_lo);
    std::swap(P->inst_hi, Q->inst_hi);
    P->total_leaves = Q->total_leaves;
    P->tables_dirty = true;
    rs_plan_destroy(Q);
    return RS_OK;
}

rs_status rs_plan_workspace_size(rs_plan P, size_t *bytes) {
    if (!P || !bytes) return RS_ERR_ARG;
    *bytes = P->total;
    return RS_OK;
}

rs_status rs_plan_destroy(rs_plan P) {
    if (!P) return RS_ERR_ARG;
    for (int i = 0; i < RING; ++i) {
        if (P->ev[i]) {
            (void)hipEventSynchronize(P->ev[i]);
            (void)hipEventDestroy(P->ev[i]);
        }
        if (P->pinned_probs[i]) (void)hipHostFree(P->pinned_probs[i]);
    }
    if (P->pinned_tables) (void)hipHostFree(P->pinned_tables);
    if (P->tables_ev) {
        (void)hipEventSynchronize(P->tables_ev);
        (void)hipEventDestroy(P->tables_ev);
    }
    for (auto &r : P->recs) {
        (void)hipEventSynchronize(r.b);
        P->pool.push_back(r.a);
        P->pool.push_back(r.b);
    }
    for (auto e : P->pool) (void)hipEventDestroy(e);
    delete P;
    return RS_OK;
}

int64_t rs_plan_query(rs_plan P, int32_t key) {
    if (!P) return -1;
    int64_t v = 0;
    switch (key) {
    case 0:
        for (auto &g : P->groups) v += (int64_t)g.leaves.size();
        return v;
    case 1:
        for (auto &g : P->groups) v += (int64_t)g.items.size();
        return v;
    case 2:
        for (auto &g : P->groups) v = std::max<int64_t>(v, g.max_depth);
        return v;
    case 3: return P->Ns;
    case 4: return P->branch;
    case 5: return P->prec;
    case 6: return P->last_refine;
    default: return -1;
    }
}

// Export the plan tables for host-side inspection: what = 0 -> leaves as
// 7 int64 per leaf (inst, t0, len, flags, slot, scratch, group); what = 1 ->
// tree items as 11 int64 per item (kind, inst, level, first, count, last,
// term_slot, out_slot, dep_first, dep_count, group).  Returns the number of
// rows (written only if cap is large enough), -1 on bad arguments.
int64_t rs_plan_export(rs_plan P, int32_t what, int64_t *out, int64_t cap_rows) {
    if (!P || (what != 0 && what != 1)) return -1;
    int64_t rows = 0;
    for (auto &g : P->groups) rows += what == 0 ? (int64_t)g.leaves.size() : (int64_t)g.items.size();
    if (!out || cap_rows < rows) return rows;
    int64_t r = 0;
    for (size_t gi = 0; gi < P->groups.size(); ++gi) {
        auto &g = P->groups[gi];
        if (what == 0) {
            for (auto &l : g.leaves) {
                int64_t *o = out + 7 * r++;
                o[0] = l.inst; o[1] = l.t0; o[2] = l.len; o[3] = l.flags; o[4] = l.slot;
                o[5] = l.scratch; o[6] = (int64_t)gi;
            }
        } else {
            for (auto &t : g.items) {
                int64_t *o = out + 11 * r++;
                o[0] = t.kind; o[1] = t.inst; o[2] = t.level; o[3] = t.first; o[4] = t.count;
                o[5] = t.last; o[6] = t.term_slot; o[7] = t.out_slot; o[8] = t.dep_first;
                o[9] = t.dep_count; o[10] = (int64_t)gi;
            }
        }
    }
    return rows;
}

static rs_status bind_and_upload(rs_plan P, const rs_problem *probs, char *work, hipStream_t st) {
    hipError_t e;
    // problem descriptors: upload only when they changed since the last call
    if (!staging_ready(P)) alloc_staging(P);
    if (!staging_ready(P)) return RS_ERR_HIP;
    std::vector<DevProb> &dp = P->dp_host;
    for (int i = 0; i < P->count; ++i) {
        const rs_problem &q = probs[i];
        DevProb &d = dp[i];
        std::memset(&d, 0, sizeof(d));
        d.Qx = q.Qx; d.Qw = q.Qw; d.Qxw = q.Qxw; d.A = q.A; d.B = q.B; d.QxN = q.QxN;
        d.x0 = q.x0; d.a = q.a; d.lx = q.lx; d.lw = q.lw; d.c = q.c; d.lN = q.lN; d.cN = q.cN;
        d.x = q.x; d.w = q.w; d.lam = q.lam; d.obj = q.obj;
        d.sQx = q.sQx; d.sQw = q.sQw; d.sQxw = q.sQxw; d.sA = q.sA; d.sB = q.sB;
        d.sa = q.sa; d.slx = q.slx; d.slw = q.slw; d.sc = q.sc;
        d.nx = q.nx; d.nu = q.nu; d.N = q.N; d.flags = q.flags;
    }
    // padded instances: the kernels see the padded copies (rs_pad.hip)
    std::vector<PadArgs> &pads = P->pads_host;
    pads.clear();
    for (int i : P->pad_inst) {
        const rs_problem &q = probs[i];
        DevProb &d = dp[i];
        const int64_t nx = q.nx, np = PAD_NU, N = q.N;
        double *b = reinterpret_cast<double *>(work + P->off_pad[i]);
        PadArgs a{};
        a.B = q.B; a.Qw = q.Qw; a.Qxw = q.Qxw; a.lw = q.lw;
        a.sB = q.sB; a.sQw = q.sQw; a.sQxw = q.sQxw; a.slw = q.slw;
        a.Bp = b;
        a.Qxwp = b + N * nx * np;
        a.Qwp = b + 2 * N * nx * np;
        a.lwp = a.Qwp + N * np * np;
        a.wp = a.lwp + N * np;
        a.sBp = q.sB ? nx * np : 0;
        a.sQxwp = q.sQxw ? nx * np : 0;
        a.sQwp = q.sQw ? np * np : 0;
        a.slwp = q.slw ? np : 0;
        a.w = q.w;
        a.nx = q.nx; a.nu = q.nu; a.nup = PAD_NU; a.N = q.N; a.flags = q.flags;
        pads.push_back(a);
        d.B = a.Bp; d.sB = a.sBp;
        d.Qw = a.Qwp; d.sQw = a.sQwp;
        d.Qxw = q.Qxw ? a.Qxwp : nullptr; d.sQxw = a.sQxwp;
        d.lw = q.lw ? a.lwp : nullptr; d.slw = a.slwp;
        d.w = a.wp;
        d.nu = PAD_NU;
    }
    if (P->refine_ws) {
        // correction problems: the same matrices; right-hand side and
        // solution in the workspace (c = cN = 0, no objective)
        for (int i = 0; i < P->count; ++i) {
            DevProb d = dp[i];
            const size_t nx = d.nx, nu = d.nu, N = d.N;
            double *b = reinterpret_cast<double *>(work + P->off_cbuf[i]);
            d.x0 = b;
            d.a = b + nx;
            d.lx = b + nx + N * nx;
            d.lw = b + nx + 2 * N * nx;
            d.lN = b + nx + 2 * N * nx + N * nu;
            d.c = nullptr;
            d.cN = nullptr;
            d.sa = nx;
            d.slx = nx;
            d.slw = nu;
            d.sc = 0;
            d.x = b + 2 * nx + 2 * N * nx + N * nu;
            d.w = d.x + (N + 1) * nx;
            d.lam = d.w + N * nu;
            d.obj = nullptr;
            dp[P->count + i] = d;
        }
    }
    const size_t nprob = dp.size();
    const bool rebind = P->bound_work != work;
    if ((rebind || P->tables_dirty) && P->tables_bytes) {
        if (hipEventSynchronize(P->tables_ev) != hipSuccess) return RS_ERR_HIP;   // the last upload has read it
        std::memcpy(P->pinned_tables, P->tables.data(), P->tables_bytes);
        e = hipMemcpyAsync(work + P->off_tables, P->pinned_tables, P->tables_bytes, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return RS_ERR_HIP;
        if (hipEventRecord(P->tables_ev, st) != hipSuccess) return RS_ERR_HIP;
        P->tables_dirty = false;
    }
    if (rebind) {
        for (auto &g : P->groups) {
            e = launch_fill_i32(reinterpret_cast<int32_t *>(work + g.off_flags),
                                (int64_t)std::max<size_t>(1, g.items.size()), 0, st);
            if (e != hipSuccess) return RS_ERR_HIP;
        }
        P->epoch = 0;
        P->probs_valid = false;
        P->bound_work = work;
    }
    // descriptors and padding jobs are one contiguous upload
    const size_t pbytes = sizeof(DevProb) * nprob, abytes = sizeof(PadArgs) * pads.size();
    if (!P->probs_valid || std::memcmp(dp.data(), P->last_probs.data(), pbytes) != 0 ||
        (abytes && std::memcmp(pads.data(), P->last_pads.data(), abytes) != 0)) {
        const int r = P->ring;
        P->ring = (P->ring + 1) % RING;
        if (P->ev_used[r] && hipEventSynchronize(P->ev[r]) != hipSuccess) return RS_ERR_HIP;
        std::memcpy(P->pinned_probs[r], dp.data(), pbytes);
        if (abytes) std::memcpy(static_cast<char *>(P->pinned_probs[r]) + pbytes, pads.data(), abytes);
        e = hipMemcpyAsync(work + P->off_probs, P->pinned_probs[r], pbytes + abytes, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return RS_ERR_HIP;
        if (hipEventRecord(P->ev[r], st) != hipSuccess) return RS_ERR_HIP;
        P->ev_used[r] = true;
        P->last_probs = dp;
        P->last_pads = pads;
        P->probs_valid = true;
    }
    return RS_OK;
}

static rs_status check_call(rs_plan P, const rs_problem *probs, void *work, size_t work_bytes) {
    if (!P || !probs || !work) return RS_ERR_ARG;
    if (work_bytes < P->total) return RS_ERR_NOMEM;
    if (reinterpret_cast<uintptr_t>(work) % ALIGN) return RS_ERR_ARG;
    for (int i = 0; i < P->count; ++i) {
        const rs_problem &q = probs[i];
        const int nu = P->nu_user[i] ? P->nu_user[i] : P->dims[3 * i + 1];
        if (q.nx != P->dims[3 * i] || q.nu != nu || q.N != P->dims[3 * i + 2]) return RS_ERR_ARG;
        if (!valid_ptr_set(q)) return RS_ERR_ARG;
        if (q.sQx < 0 || q.sQw < 0 || q.sQxw < 0 || q.sA < 0 || q.sB < 0) return RS_ERR_ARG;
        if (q.sa < 0 || q.slx < 0 || q.slw < 0 || q.sc < 0) return RS_ERR_ARG;
    }
    return RS_OK;
}

// Launch arguments of one shape group.  corr = true points the problem
// array at the correction problems of a mixed-precision plan.
static GroupArgs group_args(rs_plan P, char *W, size_t gi, int32_t *info, bool corr, bool with_conv,
                            int iter = -1) {
    Group &g = P->groups[gi];
    GroupArgs a{};
    const DevProb *user = reinterpret_cast<const DevProb *>(W + P->off_probs);
    a.probs = corr ? user + P->count : user;
    a.leaves = reinterpret_cast<const LeafItem *>(W + g.off_leaves);
    a.nleaves = (int32_t)g.leaves.size();
    a.items = reinterpret_cast<const TreeItem *>(W + g.off_items);
    a.nitems = (int32_t)g.items.size();
    a.slots = reinterpret_cast<double *>(W + g.off_slots);
    a.leaf_scratch = W + g.off_scratch;
    a.flags = reinterpret_cast<int32_t *>(W + g.off_flags);
    a.queue = reinterpret_cast<int32_t *>(W + P->off_queues) + gi;
    a.info = info;
    a.epoch = P->epoch;
    a.sps = g.shape->scratch_per_stage;
    a.ntop = g.ntop;
    a.fstore = P->factored ? W + g.off_fstore : nullptr;
    a.fvec = P->factored ? reinterpret_cast<double *>(W + g.off_fvec) : nullptr;
    a.lbw = (g.shape->lb && P->factored) ? W + g.off_lbw : nullptr;
    a.lbw_unit = (int64_t)g.lbw_unit;
    a.m1cache = P->receding ? reinterpret_cast<double *>(W + g.off_m1) : nullptr;
    a.ident = P->rank_reveal ? reinterpret_cast<const double *>(W + g.off_ident) : nullptr;
    a.nx = g.nx;
    a.nu = g.nu;
    a.superpose = P->superpose ? 1 : 0;
    if (P->refine_ws) {
        a.corr = user + P->count;
        a.conv = with_conv ? reinterpret_cast<const int32_t *>(W + P->off_conv) : nullptr;
        a.active = iter >= 0 ? reinterpret_cast<const int32_t *>(W + P->off_conv) + P->count + iter : nullptr;
        a.part = reinterpret_cast<double *>(W + P->off_part);
        a.leaf_base = g.leaf_base;
    }
    return a;
}

// One pass (leaf up, tree, leaf down) over every shape group, after a reset
// of the tree work queues (and, unless keep_status, of the status words).
// pass 0 = fused solve, 1 = stored factorization, 2 = solve on the stored
// factorization.
static rs_status launch_pass(rs_plan P, char *W, int32_t *info, hipStream_t st, int pass, bool keep_status,
                             bool corr, bool with_conv, int iter = -1) {
    static const int kinds[3][3] = {{KK_LEAF_UP, KK_TREE, KK_LEAF_DOWN},
                                    {KK_F_LEAF_UP, KK_F_TREE, KK_F_LEAF_DOWN},
                                    {KK_S_LEAF_UP, KK_S_TREE, KK_S_LEAF_DOWN}};
    ++P->epoch;
    int32_t *queues = reinterpret_cast<int32_t *>(W + P->off_queues);
    const int ninfo = keep_status ? 0 : P->count;
    hipError_t e = timed(P, KK_INIT, st, [&] { return launch_init(info, ninfo, queues, (int)P->groups.size(), st); });
    if (e != hipSuccess) return RS_ERR_HIP;
    const int f32 = P->mixed ? 1 : 0, fac = P->bf16 ? 2 : f32;
    for (size_t gi = 0; gi < P->groups.size(); ++gi) {
        Group &g = P->groups[gi];
        GroupArgs a = group_args(P, W, gi, info, corr, with_conv, iter);
        const Launcher *L = pass == 0 ? g.shape->fp64 : pass == 1 ? g.shape->factor[fac] : g.shape->vsolve[f32];
        // the vector passes run one wavefront per work item
        const int cap = pass == 2 ? 1024 : 256;
        const int tree_grid = std::max(1, std::min<int>((int)g.items.size(), cap));
        if (a.nleaves > 0) {
            e = timed(P, kinds[pass][0], st, [&] { return L[0](a, a.nleaves, st); });
            if (e != hipSuccess) return RS_ERR_HIP;
        }
        if (a.nitems > 0) {
            e = timed(P, kinds[pass][1], st, [&] { return L[1](a, tree_grid, st); });
            if (e != hipSuccess) return RS_ERR_HIP;
        }
        if (a.nleaves > 0) {
            e = timed(P, kinds[pass][2], st, [&] { return L[2](a, a.nleaves, st); });
            if (e != hipSuccess) return RS_ERR_HIP;
        }
    }
    return RS_OK;
}

// Per-leaf refinement kernel (0 residual, 1 update) over every group.
static rs_status launch_refine(rs_plan P, char *W, int32_t *info, hipStream_t st, int which, bool with_conv) {
    for (size_t gi = 0; gi < P->groups.size(); ++gi) {
        Group &g = P->groups[gi];
        GroupArgs a = group_args(P, W, gi, info, false, with_conv);
        if (a.nleaves == 0) continue;
        hipError_t e = timed(P, which == 0 ? KK_RESIDUAL : KK_UPDATE, st,
                             [&] { return g.shape->refine[which](a, a.nleaves, st); });
        if (e != hipSuccess) return RS_ERR_HIP;
    }
    return RS_OK;
}

static rs_status launch_check(rs_plan P, char *W, int32_t *info, hipStream_t st, int mode, int iter = -1) {
    int32_t *conv = reinterpret_cast<int32_t *>(W + P->off_conv);
    hipError_t e = timed(P, KK_CHECK, st, [&] {
        return launch_refine_check(reinterpret_cast<const InstInfo *>(W + P->off_inst), P->count,
                                   reinterpret_cast<const double *>(W + P->off_part),
                                   reinterpret_cast<double *>(W + P->off_stats), conv, info,
                                   reinterpret_cast<const DevProb *>(W + P->off_probs), mode, P->tol,
                                   iter >= 0 ? conv + P->count + iter : (mode == 0 ? conv + P->count : nullptr),
                                   mode == 0 ? P->max_refine + 1 : 0, P->report ? 1 : 0, st);
    });
    return e == hipSuccess ? RS_OK : RS_ERR_HIP;
}

// Infinity norm of every leaf's rows of the KKT matrix (report plans), taken
// once per factorization: the matrices do not change between its solves.
static rs_status launch_knorm_all(rs_plan P, char *W, int32_t *info, hipStream_t st) {
    for (size_t gi = 0; gi < P->groups.size(); ++gi) {
        GroupArgs a = group_args(P, W, gi, info, false, false);
        if (a.nleaves == 0) continue;
        if (timed(P, KK_REPORT, st, [&] { return launch_knorm(a, st); }) != hipSuccess) return RS_ERR_HIP;
    }
    return RS_OK;
}

// Report of an FP64 solve (report plans): the FP64 residual of the returned
// solution (relative residual, backward error), then one correction solve
// of K d = r - K z with the plan's own kernels, measured but not applied:
// ||d|| / ||z|| estimates the relative forward error of z.
static rs_status report_fp64(rs_plan P, char *W, int32_t *info, hipStream_t st, int pass) {
    rs_status s = launch_check(P, W, info, st, 0);
    if (s == RS_OK) s = launch_refine(P, W, info, st, 0, true);
    if (s == RS_OK) s = launch_check(P, W, info, st, 4);
    if (pass < 0) return s;      // leaf-chunked plans: no correction solve (est_fwd_err stays -1)
    if (s == RS_OK) s = launch_pass(P, W, info, st, pass, true, true, true);
    if (s == RS_OK) {
        for (size_t gi = 0; gi < P->groups.size() && s == RS_OK; ++gi) {
            Group &g = P->groups[gi];
            GroupArgs a = group_args(P, W, gi, info, false, true);
            a.measure_only = 1;
            if (a.nleaves == 0) continue;
            if (timed(P, KK_UPDATE, st, [&] { return g.shape->refine[1](a, a.nleaves, st); }) != hipSuccess)
                s = RS_ERR_HIP;
        }
    }
    if (s == RS_OK) s = launch_check(P, W, info, st, 5);
    return s;
}

// Solve on the stored mixed-precision factorization with FP64 iterative
// refinement: z = solve(r); then, per instance until it converges and at
// most max_refine times: rho = r - K z and the objective (FP64), convergence
// test, d = solve(rho), z += d.  Converged instances skip every later pass.
static rs_status mixed_solve(rs_plan P, char *W, int32_t *info, hipStream_t st) {
    rs_status s = launch_check(P, W, info, st, 0);
    if (s == RS_OK) s = launch_pass(P, W, info, st, 2, true, false, true);
    for (int k = 0; k < P->max_refine && s == RS_OK; ++k) {
        s = launch_refine(P, W, info, st, 0, true);
        if (s == RS_OK) s = launch_check(P, W, info, st, 1, k);     // counts active[k]
        if (s == RS_OK) s = launch_pass(P, W, info, st, 2, true, true, true, k);
        if (s == RS_OK) s = launch_refine(P, W, info, st, 1, true);
        if (s == RS_OK) s = launch_check(P, W, info, st, 2);
    }
    if (s == RS_OK) s = launch_refine(P, W, info, st, 0, true);
    if (s == RS_OK) s = launch_check(P, W, info, st, 1);
    if (s == RS_OK) s = launch_check(P, W, info, st, 3);
    P->last_refine = P->max_refine;
    return s;
}

static rs_status run_sequence(rs_plan P, char *W, int32_t *info, hipStream_t st, int mode);

// FP64 large-block solve with the leaves in chunks of P->leaf_chunk, whose
// stored factorization holds one chunk's records at a time.  Up: per chunk
// the matrix lines (records, M1 matrix part) and at once the vector lines
// on them (M1 vector part); then the master levels (matrix, then vector).
// Down: per chunk the leaf factorization again (Alg. 6 solves every leaf
// subproblem again with its parent's message; the records come out the
// same, the M1 fields they rewrite too), its vector lines and the forward
// sweep with the parent's message.  Twice the leaf matrix work of the
// stored path for a factor store bounded by one chunk.
static rs_status chunked_solve(rs_plan P, char *W, int32_t *info, hipStream_t st) {
    int32_t *queues = reinterpret_cast<int32_t *>(W + P->off_queues);
    auto chunk_args = [&](size_t gi, size_t lo, size_t hi) {
        Group &g = P->groups[gi];
        GroupArgs a = group_args(P, W, gi, info, false, false);
        a.leaves += lo;
        a.nleaves = (int32_t)(hi - lo);
        a.leaf_base += (int32_t)lo;
        a.rec_stage0 = g.leaves[lo].scratch / g.shape->scratch_per_stage;
        return a;
    };
    auto for_chunks = [&](size_t gi, auto body) -> rs_status {
        Group &g = P->groups[gi];
        for (size_t lo = 0; lo < g.leaves.size(); lo += (size_t)P->leaf_chunk) {
            const size_t hi = std::min(g.leaves.size(), lo + (size_t)P->leaf_chunk);
            rs_status s = body(chunk_args(gi, lo, hi));
            if (s != RS_OK) return s;
        }
        return RS_OK;
    };
    auto run = [&](int kind, Launcher L, const GroupArgs &a, int grid) -> rs_status {
        return timed(P, kind, st, [&] { return L(a, grid, st); }) == hipSuccess ? RS_OK : RS_ERR_HIP;
    };
    ++P->epoch;
    if (timed(P, KK_INIT, st, [&] { return launch_init(info, P->count, queues, (int)P->groups.size(), st); }) !=
        hipSuccess)
        return RS_ERR_HIP;
    for (size_t gi = 0; gi < P->groups.size(); ++gi) {
        Group &g = P->groups[gi];
        const Launcher *F = g.shape->factor[0], *V = g.shape->vsolve[0];
        rs_status s = for_chunks(gi, [&](const GroupArgs &a) {
            rs_status r = run(KK_F_LEAF_UP, F[0], a, a.nleaves);
            return r == RS_OK ? run(KK_S_LEAF_UP, V[0], a, a.nleaves) : r;
        });
        if (s != RS_OK) return s;
        if (!g.items.empty()) {
            GroupArgs a = group_args(P, W, gi, info, false, false);
            s = run(KK_F_TREE, F[1], a, std::max(1, std::min<int>((int)g.items.size(), 256)));
            if (s != RS_OK) return s;
        }
    }
    ++P->epoch;
    if (timed(P, KK_INIT, st, [&] { return launch_init(info, 0, queues, (int)P->groups.size(), st); }) !=
        hipSuccess)
        return RS_ERR_HIP;
    for (size_t gi = 0; gi < P->groups.size(); ++gi) {
        Group &g = P->groups[gi];
        if (g.items.empty()) continue;
        GroupArgs a = group_args(P, W, gi, info, false, false);
        rs_status s = run(KK_S_TREE, g.shape->vsolve[0][1], a, std::max(1, std::min<int>((int)g.items.size(), 1024)));
        if (s != RS_OK) return s;
    }
    for (size_t gi = 0; gi < P->groups.size(); ++gi) {
        Group &g = P->groups[gi];
        const Launcher *F = g.shape->factor[0], *V = g.shape->vsolve[0];
        rs_status s = for_chunks(gi, [&](const GroupArgs &a) {
            rs_status r = run(KK_F_LEAF_UP, F[0], a, a.nleaves);
            if (r == RS_OK) r = run(KK_F_LEAF_DOWN, F[2], a, a.nleaves);
            if (r == RS_OK) r = run(KK_S_LEAF_UP, V[0], a, a.nleaves);
            return r == RS_OK ? run(KK_S_LEAF_DOWN, V[2], a, a.nleaves) : r;
        });
        if (s != RS_OK) return s;
    }
    return RS_OK;
}

// The call's kernels, between the padded copies of the inputs of padded
// instances and the copy of their w back to the caller.
static rs_status run_padded(rs_plan P, char *W, int32_t *info, hipStream_t st, int mode) {
    const int npad = (int)P->pad_inst.size();
    const PadArgs *pa = reinterpret_cast<const PadArgs *>(W + P->off_padargs);
    if (npad && launch_pad(pa, npad, false, st) != hipSuccess) return RS_ERR_HIP;
    rs_status s = run_sequence(P, W, info, st, mode);
    if (s == RS_OK && npad && mode != 1 && launch_pad(pa, npad, true, st) != hipSuccess) s = RS_ERR_HIP;
    if (s == RS_OK && P->check_inputs) {
        // after the solve, so that its status words are what this overrides
        int32_t *first = reinterpret_cast<int32_t *>(W + P->off_scan);
        if (launch_fill_i32(first, P->count, 0x7fffffff, st) != hipSuccess) return RS_ERR_HIP;
        for (size_t gi = 0; gi < P->groups.size(); ++gi) {
            GroupArgs a = group_args(P, W, gi, info, false, false);
            if (timed(P, KK_REPORT, st, [&] { return launch_scan(a, first, st); }) != hipSuccess) return RS_ERR_HIP;
        }
        if (launch_scan_mark(P->count, first, info, st) != hipSuccess) return RS_ERR_HIP;
    }
    return s;
}

// Kernel sequence of a call once the descriptors are bound.
// mode 0 = rs_batch_solve, 1 = rs_factor, 2 = rs_solve.
static rs_status run_sequence(rs_plan P, char *W, int32_t *info, hipStream_t st, int mode) {
    if (P->leaf_chunk > 0) {
        rs_status s = chunked_solve(P, W, info, st);
        if (s != RS_OK || !P->report) return s;
        s = launch_knorm_all(P, W, info, st);
        return s == RS_OK ? report_fp64(P, W, info, st, -1) : s;
    }
    if (!P->mixed) {
        rs_status s;
        int solve_pass;
        if (P->via_factor && mode == 0) {
            s = launch_pass(P, W, info, st, 1, false, false, false);
            if (s == RS_OK) s = launch_pass(P, W, info, st, 2, true, false, false);
            solve_pass = 2;
        } else {
            s = launch_pass(P, W, info, st, mode, mode == 2, false, false);
            solve_pass = mode;
        }
        if (s != RS_OK || !P->report) return s;
        if (mode != 2) s = launch_knorm_all(P, W, info, st);
        if (s != RS_OK || mode == 1) return s;
        return report_fp64(P, W, info, st, solve_pass);
    }
    if (mode != 2) {
        rs_status s = launch_pass(P, W, info, st, 1, false, false, false);
        if (s == RS_OK && P->report) s = launch_knorm_all(P, W, info, st);
        if (s != RS_OK || mode == 1) return s;
    }
    return mixed_solve(P, W, info, st);
}

static rs_status run_call(rs_plan P, const rs_problem *probs, void *work, size_t work_bytes, void *stream,
                          int32_t *info_dev, int mode) {
    Range range(mode == 0 ? "rs_batch_solve" : mode == 1 ? "rs_factor" : "rs_solve");
    rs_status s = check_call(P, probs, work, work_bytes);
    if (s != RS_OK) return s;
    if (mode != 0 && (!P->factored || P->leaf_chunk > 0)) return RS_ERR_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char *W = static_cast<char *>(work);
    s = bind_and_upload(P, probs, W, st);
    if (s != RS_OK) return s;
    int32_t *info = info_dev ? info_dev : reinterpret_cast<int32_t *>(W + P->off_info);
    return run_padded(P, W, info, st, mode);
}

struct rs_graph_s {
    rs_plan plan = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

rs_status rs_graph_create(rs_plan P, int32_t mode, const rs_problem *probs, void *work, size_t work_bytes,
                          void *stream, int32_t *info_dev, rs_graph *out) {
    if (!out || mode < 0 || mode > 2 || !stream) return RS_ERR_ARG;
    *out = nullptr;
    rs_status s = check_call(P, probs, work, work_bytes);
    if (s != RS_OK) return s;
    if (mode != 0 && (!P->factored || P->leaf_chunk > 0)) return RS_ERR_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char *W = static_cast<char *>(work);
    s = bind_and_upload(P, probs, W, st);
    if (s != RS_OK) return s;
    int32_t *info = info_dev ? info_dev : reinterpret_cast<int32_t *>(W + P->off_info);
    rs_graph_s *G = new (std::nothrow) rs_graph_s();
    if (!G) return RS_ERR_NOMEM;
    G->plan = P;
    const bool timing = P->timing;
    P->timing = false;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        P->timing = timing;
        delete G;
        return RS_ERR_HIP;
    }
    // the tree flags are cleared at the start of every replay, so the epochs
    // recorded in the graph are fresh each time (a fill kernel, not a memset)
    for (auto &g : P->groups) {
        if (s == RS_OK && launch_fill_i32(reinterpret_cast<int32_t *>(W + g.off_flags),
                                          (int64_t)std::max<size_t>(1, g.items.size()), 0, st) != hipSuccess)
            s = RS_ERR_HIP;
    }
    if (s == RS_OK) s = run_padded(P, W, info, st, mode);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    P->timing = timing;
    if (s == RS_OK && (ec != hipSuccess || !graph)) s = RS_ERR_HIP;
    if (s == RS_OK && hipGraphInstantiate(&G->exec, graph, nullptr, nullptr, 0) != hipSuccess) s = RS_ERR_HIP;
    G->graph = graph;
    if (s != RS_OK) {
        if (G->exec) (void)hipGraphExecDestroy(G->exec);
        if (G->graph) (void)hipGraphDestroy(G->graph);
        delete G;
        return s;
    }
    *out = G;
    return RS_OK;
}

rs_status rs_graph_launch(rs_graph G, void *stream) {
    if (!G || !G->exec) return RS_ERR_ARG;
    return hipGraphLaunch(G->exec, reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? RS_OK : RS_ERR_HIP;
}

rs_status rs_graph_destroy(rs_graph G) {
    if (!G) return RS_ERR_ARG;
    if (G->exec) (void)hipGraphExecDestroy(G->exec);
    if (G->graph) (void)hipGraphDestroy(G->graph);
    delete G;
    return RS_OK;
}

rs_status rs_batch_solve(rs_plan P, const rs_problem *probs, void *work, size_t work_bytes, void *stream,
                         int32_t *info_dev) {
    return run_call(P, probs, work, work_bytes, stream, info_dev, 0);
}

static_assert(RS_NOALLOC_SCRATCH_BYTES == STATIC_SCRATCH_BYTES, "scratch size in rs.h and the library agree");

rs_status rs_batch_solve_noalloc(rs_plan P, const rs_problem *probs, void *stream, int32_t *info_dev) {
    if (!P || !probs) return RS_ERR_ARG;
    if (P->receding) return RS_ERR_ARG;      // its stored factors would not survive other calls' use
    size_t bytes = 0;
    void *work = static_scratch(&bytes);
    if (!work) return RS_ERR_HIP;
    if (P->total > bytes) return RS_ERR_NOMEM;
    if (!staging_ready(P)) return RS_ERR_HIP;  // plan created without a device
    // the scratch is shared by every call on this device and keeps the last
    // call's contents: bind it afresh, which uploads the tables and the
    // descriptors and clears the tree's completion flags with a fill kernel
    P->bound_work = nullptr;
    const bool timing = P->timing;            // per-kernel events would be created
    P->timing = false;
    const rs_status s = run_call(P, probs, work, bytes, stream, info_dev, 0);
    P->timing = timing;
    return s;
}

rs_status rs_refine_stats(rs_plan P, const void *work, double *out, void *stream) {
    if (!P || !work || !out) return RS_ERR_ARG;
    if (!P->mixed) return RS_ERR_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const char *W = static_cast<const char *>(work);
    // the whole statistics block, then the public columns (a plain copy:
    // the caller's buffer is ordinary host memory)
    std::vector<double> all((size_t)ST_N * P->count);
    if (hipMemcpyAsync(all.data(), W + P->off_stats, sizeof(double) * all.size(), hipMemcpyDeviceToHost, st) !=
        hipSuccess)
        return RS_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return RS_ERR_HIP;
    for (int i = 0; i < P->count; ++i)
        for (int q = 0; q < ST_PUBLIC; ++q) out[(size_t)i * ST_PUBLIC + q] = all[(size_t)i * ST_N + q];
    return RS_OK;
}

rs_status rs_info_report(rs_plan P, const void *work, const int32_t *info_dev, rs_info *report_dev, void *stream) {
    static_assert(sizeof(rs_info) == 40, "rs_info layout (3 doubles, 4 int32)");
    if (!P || !work || !report_dev) return RS_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(work) % ALIGN) return RS_ERR_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const char *W = static_cast<const char *>(work);
    const int32_t *info = info_dev ? info_dev : reinterpret_cast<const int32_t *>(W + P->off_info);
    const double *stats = P->refine_ws ? reinterpret_cast<const double *>(W + P->off_stats) : nullptr;
    return launch_report(P->count, stats, info, P->mixed ? 1 : 0, report_dev, st) == hipSuccess ? RS_OK
                                                                                                : RS_ERR_HIP;
}

rs_status rs_plan_set_timing(rs_plan P, int32_t enable) {
    if (!P) return RS_ERR_ARG;
    P->timing = enable != 0;
    return RS_OK;
}

rs_status rs_plan_kernel_times(rs_plan P, double *ms, int64_t *launches, int32_t reset) {
    if (!P || !ms || !launches) return RS_ERR_ARG;
    for (int k = 0; k < KK_COUNT; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (auto &r : P->recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) return RS_ERR_HIP;
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return RS_ERR_HIP;
        ms[r.kind] += t;
        launches[r.kind] += 1;
    }
    if (reset) {
        for (auto &r : P->recs) {
            P->pool.push_back(r.a);
            P->pool.push_back(r.b);
        }
        P->recs.clear();
    }
    return RS_OK;
}

rs_status rs_factor(rs_plan P, const rs_problem *probs, void *work, size_t work_bytes, void *stream,
                    int32_t *info_dev) {
    return run_call(P, probs, work, work_bytes, stream, info_dev, 1);
}

rs_status rs_solve(rs_plan P, const rs_problem *probs, void *work, size_t work_bytes, void *stream,
                   int32_t *info_dev) {
    return run_call(P, probs, work, work_bytes, stream, info_dev, 2);
}

}  // extern "C"
