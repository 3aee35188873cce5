// k_cussen.hip -- Cussen PC-MM (Alg. 3 with Alg. 2) on gfx950, for one
// problem (pcmm_cussen) or a compiled plan of up to 64 problems (pcmm_plan_*).
//
// Every run queues the same kernels whatever the number of problems; each
// kernel finds the problem of its block (or tile) by a binary search over the
// per-problem prefix offsets held in the descriptors of the plan image:
//   table_build   one lane per (problem, unit = column k of A, J output
//                 columns j, point): runs the column's straight-line program
//                 (level-N ladders, prefix sums) on B[k, j], keeps every
//                 register in a lane-private scratch (structure of arrays, so
//                 the lanes' accesses coalesce), then converts its digit
//                 tables to affine with one inversion for all of its J tables.
//   coop_table    (runs with narrow problems only) the same digit tables
//                 with several lanes per level-1 chain: block sums, a scan
//                 across the lanes, one inversion per lane.
//   combo_table   (column groups g > 1) one lane per (group, output column j,
//                 point): the group's digit combinations, level by level, each
//                 an affine addition of two entries of the table, with one
//                 batched inversion per level.
//   accumulate    persistent: workgroups take tiles (problem, row tile, pair
//                 tile, split) from a device queue, the most expensive tiles
//                 first.  For a tile, C_ij += sign * T_kj[code_ik]: every
//                 lane owns one accumulator (row i, pair) in VGPRs and walks
//                 its row's nonzero codes with mixed additions, gathering
//                 the entries from the tables in global memory (a
//                 wavefront's lanes share the pair, so L1 and L2 serve
//                 them).  The inner dimension may be split over
//                 independent partial sums.
//   reduce        adds the split-k partial sums of one output with a tree of
//                 point additions across the lanes of a wavefront (shuffles).
//   normalize     Jacobian -> canonical affine C with batched inversion.
#include <algorithm>
#include <atomic>
#include <cstddef>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "normalize.hpp"
#include "normalize_dev.hpp"
#include "plan.hpp"

using namespace pcmm;

namespace {

// Affine table entry, Montgomery form, normal limbs: an x granule and a y
// granule of NL words each.  The tables of a group hold, per entry e, an x
// plane and then a y plane of one granule per (j, point) pair, pair-fastest,
// so the lanes of a wavefront (consecutive pairs) touch one contiguous span
// per plane.  Bit 31 of x's limb 8 marks the identity (stored as x = y = 0);
// a normal-form limb 8 is below 2^25, which leaves bit 30 for the
// combination build's mark of entries it finishes in its third pass.
constexpr int ENTRY_WORDS = 2 * NL;
constexpr uint32_t ENTRY_INF = 1u << 31;
constexpr uint32_t ENTRY_PENDING = 1u << 30;
constexpr uint32_t LIMB8_BITS = ENTRY_PENDING - 1;
constexpr int JAC_WORDS = 3 * NL;
constexpr int MAX_PROBLEMS = PCMM_PLAN_MAX_PROBLEMS;
// the autotuner skips column groups g > 1 whose single (group, pair) table is
// larger than this: such a table's build would outweigh what it saves
constexpr size_t GROUP_TABLE_CAP = 150 * 1024;

// One problem of a run, as the kernels see it.  Offsets o_* are bytes into
// the plan image, w_* bytes into the workspace; the image sits at the start
// of the workspace, descriptors first.
struct prob_desc {
    int32_t m, n, l, g;
    int32_t ngroups, emax, rmax, c_form;
    int32_t J, Lj, tm, pp;
    int32_t kc, S, gps, io;  // io: index of the problem's matrices in the run
    int32_t tiles_x, tiles_y, norm_per, coop_w;  // coop_w: lanes per level-1 chain (0: one lane per chain)
    int32_t coop_lpu, coop_h;  // cooperative build: lanes per unit; first register slot of a lane's block
    int32_t nunits, levels;  // digit-table units (columns); largest combination level (1: none)
    int64_t n_lanes, tb_block0;
    int64_t cb_lanes, cb_block0;  // combination lanes (group, pair), 0 without combinations
    int64_t tile0;
    int64_t red_block0, red_threads;
    int64_t norm_block0, norm_threads;
    int64_t ldj;     // ld of the internal Jacobian buffers (partials, C before normalisation)
    int64_t ld_pre;  // ld of the normalisation prefixes
    int64_t o_ops, o_op_begin, o_entry_begin, o_entries, o_entry_value;
    int64_t o_unit_col, o_unit_grp, o_unit_off, o_cblock_begin, o_cblocks, o_cruns;
    int64_t o_lists, o_chunk_off, o_chunk_len;  // nonzero codes per (split, chunk), see pack_codes
    int32_t chunks_per_split;
    int32_t direct;  // one column group, one split, affine C: each output is one table entry
    int64_t w_regs, w_table, w_part, w_cjac, w_norm;
    int64_t w_cprod;  // combination lanes' level products and pending marks (10 planes of cb_lanes words)
};

struct io_ptrs {
    const uint32_t *B;  // n x l ciphertexts, affine canonical
    uint32_t *C;        // m x l, canonical, the problem's c_form
    int64_t ldb, ldc;
};

struct run_args {
    char *ws;            // workspace (w_* offsets)
    const char *desc;    // this launch's descriptors (in the workspace)
    const char *plan;    // base of the plan arrays (o_* offsets): the workspace, or a resident copy
    int32_t count;       // descriptors
    int32_t pad;
    int64_t total_tiles;
    int64_t ctr_off;     // byte offset of the accumulation queue counter
    io_ptrs io[MAX_PROBLEMS];
};

__device__ __forceinline__ const prob_desc *descs(const run_args &a) { return (const prob_desc *)a.desc; }

// last problem whose prefix value (the int64 at byte offset key_off of its
// descriptor) is <= x; problems with empty ranges are skipped by construction
__device__ __forceinline__ int find_problem(const run_args &a, size_t key_off, int64_t x) {
    const char *d = (const char *)descs(a);
    int lo = 0, hi = a.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t k = *(const int64_t *)(d + (size_t)mid * sizeof(prob_desc) + key_off);
        if (k <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename T>
__device__ __forceinline__ T *at(const run_args &a, int64_t off) {
    return (T *)(a.ws + off);
}

template <typename T>
__device__ __forceinline__ const T *plan_at(const run_args &a, int64_t off) {
    return (const T *)(a.plan + off);
}

// --------------------------------------------------------------------------
// Table entries
// --------------------------------------------------------------------------
// 16-byte access at a 4-byte aligned address (a granule starts at 36 p bytes)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4), aligned(4)));

// Words from one entry of a (group, pair) table to the next, and from an
// entry's x granule to its y granule.
__host__ __device__ __forceinline__ int64_t entry_stride(int64_t npairs) { return 2 * npairs * NL; }
__host__ __device__ __forceinline__ int64_t y_offset(int64_t npairs) { return npairs * NL; }

// x granule of entry e of group grp's table for pair p
__device__ __forceinline__ uint32_t *entry_at(uint32_t *table, int64_t npairs, int emax, int grp, int e, int64_t p) {
    return table + (((int64_t)grp * emax + e) * 2 * npairs) * NL + p * NL;
}

__device__ __forceinline__ fe load_gran(const uint32_t *g) {
    const u32x4 a = *(const u32x4 *)g;
    const u32x4 b = *(const u32x4 *)(g + 4);
    return fe{{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, g[8]}};
}

// stores v with `flags` or-ed into limb 8
__device__ __forceinline__ void store_gran(uint32_t *g, const fe &v, uint32_t flags) {
    *(u32x4 *)g = u32x4{v.v[0], v.v[1], v.v[2], v.v[3]};
    *(u32x4 *)(g + 4) = u32x4{v.v[4], v.v[5], v.v[6], v.v[7]};
    g[8] = v.v[8] | flags;
}

// x of an entry and its flag bits
__device__ __forceinline__ fe read_x(const uint32_t *slot, uint32_t &flags) {
    fe x = load_gran(slot);
    flags = x.v[8] & ~LIMB8_BITS;
    x.v[8] &= LIMB8_BITS;
    return x;
}

__device__ __forceinline__ apt read_entry(const uint32_t *slot, int64_t yoff, bool &inf) {
    uint32_t flags;
    apt A;
    A.x = read_x(slot, flags);
    A.y = load_gran(slot + yoff);
    inf = (flags & ENTRY_INF) != 0;
    return A;
}

__device__ __forceinline__ void write_entry(uint32_t *slot, int64_t yoff, const apt &A, bool inf) {
    store_gran(slot, inf ? fe_zero() : A.x, inf ? ENTRY_INF : 0u);
    store_gran(slot + yoff, inf ? fe_zero() : A.y, 0u);
}

// --------------------------------------------------------------------------
// Table build
// --------------------------------------------------------------------------
__device__ __forceinline__ jpt reg_load(const uint32_t *regs, int rmax, int64_t n_lanes, int r, int reg,
                                        int64_t lane) {
    return load_jac_m(regs + (int64_t)(r * rmax + reg) * JAC_WORDS * n_lanes, n_lanes, 0, lane);
}

__device__ __forceinline__ void reg_store(uint32_t *regs, int rmax, int64_t n_lanes, int r, int reg, int64_t lane,
                                          const jpt &P) {
    store_jac_m(regs + (int64_t)(r * rmax + reg) * JAC_WORDS * n_lanes, n_lanes, 0, lane, P);
}

// One op of a column's straight-line program for output column j, point pt
// and chain r: reads its operands (registers or the column's base point
// B[k0, j], loaded once per chain: every negative operand of a unit's
// program names it, which the plan check enforces) and writes its
// destination register.  The previous op's
// result stays in VGPRs (`last`, register `last_reg`): a prefix sum's first
// operand is the sum before it, so most operands need no reload.
__device__ __forceinline__ jpt op_reg(const uint32_t *regs, int rmax, int64_t n_lanes, int r, int reg, int64_t lane,
                                      const jpt &last, int last_reg) {
    return reg == last_reg ? last : reg_load(regs, rmax, n_lanes, r, reg, lane);
}

__device__ __forceinline__ void run_op(const plan_op op, const apt &base, uint32_t *regs, int rmax, int64_t n_lanes,
                                       int r, int64_t lane, jpt &last, int &last_reg) {
    jpt R;
    if (op.kind == OP_MUL) {
        const int s = op.s;
        const int bits = 32 - __builtin_clz((unsigned)s);
        R = ladder_small<false>((uint32_t)s, bits, base);
    } else if (op.a >= 0 && op.b >= 0) {
        jpt Q = op_reg(regs, rmax, n_lanes, r, op.b, lane, last, last_reg);
        if (op.neg_b) Q = jpt_neg(Q);
        R = jpt_add<false>(op_reg(regs, rmax, n_lanes, r, op.a, lane, last, last_reg), Q);
    } else if (op.b < 0) {
        const apt Q = op.neg_b ? apt_neg(base) : base;
        jpt P = op.a >= 0 ? op_reg(regs, rmax, n_lanes, r, op.a, lane, last, last_reg) : jpt_from_affine(base);
        R = jpt_add_affine_lean<false>(P, Q);
    } else {
        // a is the base point, b a register: a + (+-b) = (+-b) + a
        jpt Q = op_reg(regs, rmax, n_lanes, r, op.b, lane, last, last_reg);
        if (op.neg_b) Q = jpt_neg(Q);
        R = jpt_add_affine_lean<false>(Q, base);
    }
    reg_store(regs, rmax, n_lanes, r, op.dst, lane, R);
    last = R;
    last_reg = op.dst;
}

// Operand of a single-column program (a register, or the base point B_kj)
// as a Jacobian point.
__device__ __forceinline__ jpt operand_point(int16_t opd, const apt &base, const uint32_t *regs, int rmax,
                                             int64_t n_lanes, int64_t lane) {
    if (opd < 0) return jpt_from_affine(base);
    return reg_load(regs, rmax, n_lanes, 0, opd, lane);
}

__device__ __forceinline__ jpt shfl_up_jpt(const jpt &P, int delta, int width) {
    jpt R;
#pragma unroll
    for (int w = 0; w < NL; ++w) {
        R.X.v[w] = (uint32_t)__shfl_up((int)P.X.v[w], delta, width);
        R.Y.v[w] = (uint32_t)__shfl_up((int)P.Y.v[w], delta, width);
        R.Z.v[w] = (uint32_t)__shfl_up((int)P.Z.v[w], delta, width);
    }
    return R;
}

// v B for a small v >= 1: left to right, a doubling per bit below the top
// one and the mixed addition of B where the bit is set (lanes whose v is
// shorter leave the loop early: masked, unchanged)
__device__ __forceinline__ jpt small_multiple(uint32_t v, const apt &B) {
    jpt R = jpt_from_affine(B);
    for (int i = 30 - __builtin_clz(v); i >= 0; --i) {
        R = jpt_dbl<false>(R);
        const jpt T = jpt_add_affine_lean<false>(R, B);
        if ((v >> i) & 1u) R = T;
    }
    return R;
}

// Table of one (group, j, point) built by W lanes (a padded run of
// single-column groups; whole wavefronts per group, 2 l chains of W lanes).  The
// program's last E - 1 ops are the level-1 prefix sums S_i = S_{i-1} + b_i
// (S_0 = b_0), and S_i = value_i B_kj with value_i the i-th smallest
// magnitude of the column (the plan records it).  Every lane runs the ops
// before the chain (levels >= 2, a few short chains, for the b_i that are
// registers), starts its block at S_i0 = value_i0 B_kj (a short ladder), runs
// the block's prefix sums from there (storing each S_i once), then converts
// its block's entries to affine with one inversion.  Chain depth: about
// 1.5 log2(value) + E / W additions instead of E.
__device__ __forceinline__ void coop_table_build(const run_args &a, const prob_desc &d, int64_t lane) {
    const int W = d.coop_w, l = d.l, lpu = d.coop_lpu;
    // a unit's lanes are whole wavefronts: its index in a scalar register,
    // so that the program's arrays come through scalar loads
    const int u = __builtin_amdgcn_readfirstlane((int)(lane / lpu));
    const int rem = (int)(lane % lpu);
    const int chain = rem / W, w = rem % W;
    if (chain >= 2 * l) return;  // whole W-lane segments idle
    const int j = chain >> 1, pt = chain & 1;
    const plan_op *ops = plan_at<plan_op>(a, d.o_ops);
    const int32_t *op_begin = plan_at<int32_t>(a, d.o_op_begin);
    const int32_t *entry_begin = plan_at<int32_t>(a, d.o_entry_begin);
    const int16_t *entries = plan_at<int16_t>(a, d.o_entries);
    const int32_t *entry_value = plan_at<int32_t>(a, d.o_entry_value);
    uint32_t *regs = at<uint32_t>(a, d.w_regs);
    uint32_t *table = at<uint32_t>(a, d.w_table);
    const uint32_t *B = a.io[d.io].B;
    const int64_t ldb = a.io[d.io].ldb;
    const int rmax = d.rmax, emax = d.emax;
    const int64_t n_lanes = d.n_lanes;
    const int k0 = plan_at<int32_t>(a, d.o_unit_col)[u];
    const int grp = plan_at<int32_t>(a, d.o_unit_grp)[u];
    const int off = plan_at<int32_t>(a, d.o_unit_off)[u];
    const int ob = op_begin[u], oe = op_begin[u + 1];
    const int eb = entry_begin[u], E = entry_begin[u + 1] - eb;
    if (E == 0) return;  // uniform over the chain's lanes
    const int ofirst = oe - (E - 1);
    // levels >= 2, on every lane (each keeps its own register column)
    jpt last = jpt_infinity();
    int last_reg = -1;
    const apt base = load_affine(B, ldb, pt, (int64_t)k0 * l + j);
    for (int o = ob; o < ofirst; ++o) run_op(ops[o], base, regs, rmax, n_lanes, 0, lane, last, last_reg);
    // this lane's block of the chain
    const int bs = (E + W - 1) / W;
    const int i0 = min(E, w * bs), i1 = min(E, i0 + bs);
    const int64_t npairs = 2 * (int64_t)l;
    uint32_t *tab = entry_at(table, npairs, emax, grp, off, 2 * j + pt);
    const int64_t estride = entry_stride(npairs), yoff = y_offset(npairs);
    fe prod = fe_one_mont();
    jpt S = jpt_infinity();
    // (this lane's entry and chain operands are read one entry ahead, before
    // the current entry's stores: a wait for a load also waits for the
    // memory operations issued before it)
    int16_t opd_n = i0 < i1 ? entries[eb + i0] : (int16_t)-1;
    int16_t opdb_n = i0 > 0 && i0 < i1 ? ops[ofirst + i0 - 1].b : (int16_t)-1;
    for (int i = i0; i < i1; ++i) {
        const int16_t opd = opd_n, opd_b = opdb_n;
        if (i + 1 < i1) {
            opd_n = entries[eb + i + 1];
            opdb_n = ops[ofirst + i].b;
        }
        if (i == 0) {
            S = operand_point(opd, base, regs, rmax, n_lanes, lane);  // b_0, as the program made it
        } else if (i == i0) {
            S = small_multiple((uint32_t)entry_value[eb + i], base);
        } else {
            S = opd_b < 0 ? jpt_add_affine_lean<false>(S, base)
                          : jpt_add<false>(S, reg_load(regs, rmax, n_lanes, 0, opd_b, lane));
        }
        if (opd < 0) continue;  // S_0 = B_kj: affine already
        // S_0 = b_0 is its own register; a later entry goes to its slot in
        // the lane's block
        if (i > 0) reg_store(regs, rmax, n_lanes, 0, d.coop_h + (i - i0), lane, S);
        store_gran(tab + i * estride, prod, 0u);
        if (!fe_is_zero(S.Z)) prod = fe_mul_t<false, true>(prod, S.Z);
    }
    fe inv = fe_inv(prod);
    // an entry's register and stored prefix are loaded one entry ahead,
    // before the current entry's stores
    jpt nP = jpt_infinity();
    fe npre = fe_zero();
    auto fetch = [&](int i, int16_t opd) {
        if (opd >= 0) {
            nP = reg_load(regs, rmax, n_lanes, 0, i == 0 ? (int)opd : d.coop_h + (i - i0), lane);
            npre = load_gran(tab + i * estride);
        }
    };
    int16_t bo_n = i1 > i0 ? entries[eb + i1 - 1] : (int16_t)-1;
    int16_t bo_n2 = i1 - 2 >= i0 ? entries[eb + i1 - 2] : (int16_t)-1;
    if (i1 > i0) fetch(i1 - 1, bo_n);
    for (int i = i1 - 1; i >= i0; --i) {
        const int16_t opd = bo_n;
        const jpt P = nP;
        const fe pre = npre;
        if (i > i0) {
            bo_n = bo_n2;
            fetch(i - 1, bo_n);
            if (i - 2 >= i0) bo_n2 = entries[eb + i - 2];
        }
        apt A;
        if (opd < 0) {
            A = base;
        } else if (fe_is_zero(P.Z)) {
            A.x = fe_zero();
            A.y = fe_zero();
        } else {
            const fe zinv = fe_mul_t<false, true>(inv, pre);
            inv = fe_mul_t<false, true>(inv, P.Z);
            A = jpt_to_affine_with(P, zinv);
        }
        write_entry(tab + i * estride, yoff, A, apt_is_inf(A));
    }
}

// The tables of the run's problems with coop_w > 1 (launched over the same
// blocks as table_build_kernel, which skips those problems).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) coop_table_kernel(run_args a) {
    const int b = find_problem(a, offsetof(prob_desc, tb_block0), blockIdx.x);
    const prob_desc &d = descs(a)[b];
    const int64_t lane = ((int64_t)blockIdx.x - d.tb_block0) * blockDim.x + threadIdx.x;
    if (d.coop_w <= 1 || lane >= d.n_lanes) return;
    coop_table_build(a, d, lane);
}

// Two wavefronts per SIMD (<= 256 VGPRs): the kernel waits on its register
// file in HBM, and a second wavefront hides much of that latency.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) table_build_kernel(run_args a) {
    // the accumulation that follows on the stream starts its queue at zero
    if (blockIdx.x == 0 && threadIdx.x == 0) *at<int32_t>(a, a.ctr_off) = 0;
    const int b = find_problem(a, offsetof(prob_desc, tb_block0), blockIdx.x);
    const prob_desc &d = descs(a)[b];
    const int64_t lane = ((int64_t)blockIdx.x - d.tb_block0) * blockDim.x + threadIdx.x;
    if (lane >= d.n_lanes) return;
    if (d.coop_w > 1) return;  // coop_table_kernel builds this problem's tables
    const plan_op *ops = plan_at<plan_op>(a, d.o_ops);
    const int32_t *op_begin = plan_at<int32_t>(a, d.o_op_begin);
    const int32_t *entry_begin = plan_at<int32_t>(a, d.o_entry_begin);
    const int16_t *entries = plan_at<int16_t>(a, d.o_entries);
    uint32_t *regs = at<uint32_t>(a, d.w_regs);
    uint32_t *table = at<uint32_t>(a, d.w_table);
    const uint32_t *B = a.io[d.io].B;
    const int64_t ldb = a.io[d.io].ldb;
    const int l = d.l, rmax = d.rmax, emax = d.emax;
    const int64_t n_lanes = d.n_lanes;
    const int64_t npairs = 2 * (int64_t)l;
    const int64_t estride = entry_stride(npairs), yoff = y_offset(npairs);

    const int lanes_per_unit = 2 * d.Lj;
    const int u = (int)(lane / lanes_per_unit);
    const int rem = (int)(lane % lanes_per_unit);
    const int jslot = rem >> 1;
    const int pt = rem & 1;
    const int k0 = plan_at<int32_t>(a, d.o_unit_col)[u];
    const int grp = plan_at<int32_t>(a, d.o_unit_grp)[u];
    const int off = plan_at<int32_t>(a, d.o_unit_off)[u];
    const int ob = op_begin[u], oe = op_begin[u + 1];
    const int eb = entry_begin[u], ee = entry_begin[u + 1];
    const int E = ee - eb;

    fe prod = fe_one_mont();
    int last_r = -1;
    for (int r = 0; r < d.J; ++r) {
        const int j = jslot + r * d.Lj;
        if (j >= l) break;
        last_r = r;
        jpt last = jpt_infinity();
        int last_reg = -1;
        uint32_t *tab = entry_at(table, npairs, emax, grp, off, 2 * j + pt);
        const apt base = load_affine(B, ldb, pt, (int64_t)k0 * l + j);
        // forward pass of the batched inversion, folded into the program: the
        // plan orders a group's entries by their producing ops, so the next
        // register entry is always the next one an op produces, and its Z
        // joins the running product while it is still in registers (entry
        // slots hold the products before them)
        int ne = 0;
        while (ne < E && entries[eb + ne] < 0) ++ne;
        for (int o = ob; o < oe; ++o) {
            const plan_op op = ops[o];
            run_op(op, base, regs, rmax, n_lanes, r, lane, last, last_reg);
            if (ne < E && op.dst == entries[eb + ne]) {
                store_gran(tab + ne * estride, prod, 0u);
                if (!fe_is_zero(last.Z)) prod = fe_mul_t<false, true>(prod, last.Z);
                ++ne;
                while (ne < E && entries[eb + ne] < 0) ++ne;
            }
        }
    }
    if (last_r < 0) return;
    fe inv = fe_inv(prod);
    for (int r = last_r; r >= 0; --r) {
        const int j = jslot + r * d.Lj;
        uint32_t *tab = entry_at(table, npairs, emax, grp, off, 2 * j + pt);
        const apt base = load_affine(B, ldb, pt, (int64_t)k0 * l + j);
        // an entry's register and stored prefix are loaded one entry ahead,
        // before the current entry's stores (the wait for a load also waits
        // for the memory operations issued before it)
        jpt nP = jpt_infinity();
        fe npre = fe_zero();
        auto fetch = [&](int e) {
            const int16_t opd = entries[eb + e];
            if (opd >= 0) {
                nP = reg_load(regs, rmax, n_lanes, r, opd, lane);
                npre = load_gran(tab + e * estride);
            }
        };
        if (E > 0) fetch(E - 1);
        for (int e = E - 1; e >= 0; --e) {
            const int16_t opd = entries[eb + e];
            const jpt P = nP;
            const fe pre = npre;
            if (e > 0) fetch(e - 1);
            apt A;
            if (opd < 0) {
                A = base;
            } else if (fe_is_zero(P.Z)) {
                A.x = fe_zero();
                A.y = fe_zero();
            } else {
                fe zinv = fe_mul_t<false, true>(inv, pre);
                inv = fe_mul_t<false, true>(inv, P.Z);
                A = jpt_to_affine_with(P, zinv);
            }
            write_entry(tab + e * estride, yoff, A, apt_is_inf(A));
        }
    }
}

// --------------------------------------------------------------------------
// Combination entries (column groups g > 1)
// --------------------------------------------------------------------------
// a - b - c + 4p (mod p) for a, b, c normal: one limb pass (value in
// (0, 6p)), then normalised
__device__ __forceinline__ fe fe_sub_sub(const fe &a, const fe &b, const fe &c) {
    fe x;
#pragma unroll
    for (int i = 0; i < NL; ++i) x.v[i] = a.v[i] - b.v[i] - c.v[i] + (uint32_t)KP4.v[i];
    return fe_norm(x);
}

// a + b for the cases the chord formula does not cover: an identity operand,
// b = -a (the identity) and b = a (the doubling, with an inversion of its
// own; a P-256 point has no order 2, so 2a is finite).  Rare: random
// ciphertexts never meet them, forced inputs in the tests do.
__device__ __noinline__ void combo_special(const uint32_t *sa, const uint32_t *sb, int64_t yoff, bool neg_b,
                                           uint32_t *dst) {
    bool a_inf, b_inf;
    const apt A = read_entry(sa, yoff, a_inf);
    apt Bn = read_entry(sb, yoff, b_inf);
    if (neg_b) Bn.y = fe_neg(Bn.y);
    apt R = A;
    bool inf = false;
    if (a_inf && b_inf) {
        inf = true;
    } else if (a_inf) {
        R = Bn;
    } else if (b_inf) {
        R = A;
    } else if (!fe_eq(A.y, Bn.y)) {  // x equal, y opposite
        inf = true;
    } else {
        const jpt D = jpt_dbl<false>(jpt_from_affine(A));
        R = jpt_to_affine_with(D, fe_inv(D.Z));
    }
    write_entry(dst, yoff, R, inf);
}

// 4p - a - b for a, b normal: (0, 4p], carry-only (the negated second
// operand's y minus the first's in one limb pass)
__device__ __forceinline__ fe fe_neg_sub_w(const fe &a, const fe &b) {
    fe x;
#pragma unroll
    for (int i = 0; i < NL; ++i) x.v[i] = (uint32_t)KP4.v[i] - a.v[i] - b.v[i];
    fe_carry(x);
    return x;
}

// x_b - x_a of a chord: carry-only in (0, 4p) for the products, or (SAFE)
// normalised, with the chord condition x_a != x_b tested
template <bool SAFE>
__device__ __forceinline__ fe chord_dx(const fe &xb, const fe &xa, bool &ne) {
    if constexpr (SAFE) {
        const fe dx = fe_sub(xb, xa);
        ne = !fe_is_zero(dx);
        return dx;
    } else {
        ne = true;
        return fe_sub_w(xb, xa);
    }
}

// The combinations of one (group, output column j, point), lane = (group,
// pair) of the problem; the lanes of a wavefront are consecutive pairs, so
// with the plane layout of the tables their accesses to one entry's x (or y)
// are one contiguous span.  Within a level every combination reads only
// lower levels, so one inversion (Montgomery's trick) serves the whole
// level.  The level's combinations come in blocks of up to COMBO_BLOCK first
// operands a[r], held in registers, and runs of one second operand b each
// (loaded once per run):
//   forward   the product of the dx = x_b - x_a[r] of all chord additions
//             (reading only x), one prefix (the product before the run)
//             stored per run, in the x granule of its first combination;
//   inverse   one inversion per level, shared by two lanes;
//   backward  per run (in reverse) the prefixes inside the run again from
//             the run's dx, then each combination's 1/dx and its affine sum
//             by the chord formula.
// The chord formula needs two finite operands with x_a != x_b.  The first
// forward pass excludes only identity operands (flags); a pair with x_a =
// x_b then makes the level's product zero, and a wavefront with such a lane
// runs the level's forward pass again with x_a != x_b tested per
// combination (and the matching backward pass).  Combinations the chord
// formula does not cover are marked (ENTRY_PENDING in limb 8 of x) and
// finished in a third pass, which runs only when some lane of the wavefront
// has one.
constexpr int CB = COMBO_BLOCK;

// The passes' products take loose quotient digits (fp.hpp): every operand
// pair is below 16 p^2 (normal values, carry-only differences below 4p).
__device__ __forceinline__ fe fe_mul_lq(const fe &a, const fe &b) { return fe_mul_t<false, true>(a, b); }
__device__ __forceinline__ fe fe_sqr_lq(const fe &a) { return fe_sqr_t<false, true>(a); }

template <bool SAFE>
__device__ __forceinline__ fe combo_forward(const plan_cblock *blocks, const plan_crun *runs, int b0, int b1,
                                            uint32_t *tab, int64_t estride, bool &pending) {
    fe prod = fe_one_mont();
    for (int bi = b0; bi < b1; ++bi) {
        const plan_cblock blk = blocks[bi];
        fe xa[CB];
        bool ainf[CB];
#pragma unroll
        for (int r = 0; r < CB; ++r) {
            if (r < blk.na) {
                uint32_t fl;
                xa[r] = read_x(tab + blk.a[r] * estride, fl);
                ainf[r] = (fl & ENTRY_INF) != 0;
            } else {  // no such operand: an identity, never a chord
                xa[r] = fe_zero();
                ainf[r] = true;
            }
        }
        plan_crun nr = runs[blk.run_begin];
        uint32_t nfl;
        fe nxb = read_x(tab + nr.b * estride, nfl);
        for (int ri = blk.run_begin; ri < blk.run_end; ++ri) {
            const plan_crun run = nr;
            const fe xb = nxb;
            const bool binf = (nfl & ENTRY_INF) != 0;
            if (ri + 1 < blk.run_end) {
                nr = runs[ri + 1];
                nxb = read_x(tab + nr.b * estride, nfl);
            }
            // the run's product of dx first, then one product into the
            // running chain (its critical path: one product per run)
            const fe one = fe_one_mont();
            fe t = one;
            bool chord[CB];
            int first = -1;
#pragma unroll
            for (int r = 0; r < CB; ++r) {
                bool ne;
                const fe dx = chord_dx<SAFE>(xb, xa[r], ne);
                const bool present = run.dst[r] >= 0;
                chord[r] = present && !ainf[r] && !binf && ne;
                if (present && first < 0) first = r;
                if (present && !chord[r]) pending = true;
                const fe f = fe_select(chord[r], one, dx);
                t = r == 0 ? f : fe_mul_lq(t, f);
            }
#pragma unroll
            for (int r = 0; r < CB; ++r) {
                if (r == first) {
                    store_gran(tab + run.dst[r] * estride, prod, chord[r] ? 0u : ENTRY_PENDING);
                } else if (run.dst[r] >= 0 && !chord[r]) {
                    tab[run.dst[r] * estride + NL - 1] = ENTRY_PENDING;
                }
            }
            prod = fe_mul_lq(prod, t);
        }
    }
    return prod;
}

template <bool SAFE>
__device__ __forceinline__ void combo_backward(const plan_cblock *blocks, const plan_crun *runs, int b0, int b1,
                                               uint32_t *tab, int64_t estride, int64_t yoff, fe inv) {
    for (int bi = b1 - 1; bi >= b0; --bi) {
        const plan_cblock blk = blocks[bi];
        apt A[CB];
        bool ainf[CB];
#pragma unroll
        for (int r = 0; r < CB; ++r) {
            if (r < blk.na) {
                A[r] = read_entry(tab + blk.a[r] * estride, yoff, ainf[r]);
            } else {  // no such operand: an identity, never a chord
                A[r].x = fe_zero();
                A[r].y = fe_zero();
                ainf[r] = true;
            }
        }
        // a run's second operand and its stored prefix are loaded one run
        // ahead, before the current run's stores (the wait for a load also
        // waits for the memory operations issued before it)
        auto prefix_slot = [&](const plan_crun &rn) {
            int first = 0;
            while (rn.dst[first] < 0) ++first;
            return tab + rn.dst[first] * estride;
        };
        plan_crun nr = runs[blk.run_end - 1];
        bool nbinf;
        apt nb = read_entry(tab + nr.b * estride, yoff, nbinf);
        fe npre = load_gran(prefix_slot(nr));
        for (int ri = blk.run_end - 1; ri >= blk.run_begin; --ri) {
            const plan_crun run = nr;
            const apt Bv = nb;
            const bool binf = nbinf;
            fe cur = npre;
            if (ri > blk.run_begin) {
                nr = runs[ri - 1];
                nb = read_entry(tab + nr.b * estride, yoff, nbinf);
                npre = load_gran(prefix_slot(nr));
            }
            // the prefix before each combination of the run, then every
            // combination's 1/dx (newest first, the inverse chain), then
            // the chord sums; branch-free, so the run's independent chains
            // interleave (the rare non-chord slots compute discarded values
            // and are not stored)
            const fe one = fe_one_mont();
            fe q[CB], dx[CB], dinv[CB];
            bool chord[CB];
            cur.v[NL - 1] &= LIMB8_BITS;
#pragma unroll
            for (int r = 0; r < CB; ++r) {
                bool ne;
                dx[r] = chord_dx<SAFE>(Bv.x, A[r].x, ne);
                chord[r] = run.dst[r] >= 0 && !ainf[r] && !binf && ne;
                q[r] = cur;
                if (r + 1 < CB) cur = fe_mul_lq(cur, fe_select(chord[r], one, dx[r]));
            }
#pragma unroll
            for (int r = CB - 1; r >= 0; --r) {
                dinv[r] = fe_mul_lq(inv, q[r]);
                inv = fe_mul_lq(inv, fe_select(chord[r], one, dx[r]));
            }
#pragma unroll
            for (int r = 0; r < CB; ++r) {
                // y_b - y_a, or -y_b - y_a for a subtracted b: carry-only
                const fe dy = ((run.neg >> r) & 1) ? fe_neg_sub_w(Bv.y, A[r].y) : fe_sub_w(Bv.y, A[r].y);
                const fe lam = fe_mul_lq(dy, dinv[r]);
                apt R;
                R.x = fe_sub_sub(fe_sqr_lq(lam), A[r].x, Bv.x);
                R.y = fe_sub(fe_mul_lq(lam, fe_sub_w(A[r].x, R.x)), A[r].y);
                if (chord[r]) write_entry(tab + run.dst[r] * estride, yoff, R, false);
            }
        }
    }
}

// One level's blocks [b0, b1) of a combination lane's group (a group's
// blocks are ordered by level); the lane's table and strides.
struct combo_lane {
    const plan_cblock *blocks;
    const plan_crun *runs;
    uint32_t *tab;
    int64_t estride, yoff;
    int b0, b1;
};

__device__ __forceinline__ combo_lane combo_lane_of(const run_args &a, const prob_desc &d, int64_t lane, int level) {
    const int npairs = 2 * d.l;
    const int grp = (int)(lane / npairs);
    const int p = (int)(lane - (int64_t)grp * npairs);
    const int32_t *cblock_begin = plan_at<int32_t>(a, d.o_cblock_begin);
    combo_lane c;
    c.blocks = plan_at<plan_cblock>(a, d.o_cblocks);
    c.runs = plan_at<plan_crun>(a, d.o_cruns);
    c.tab = entry_at(at<uint32_t>(a, d.w_table), npairs, d.emax, grp, 0, p);
    c.estride = entry_stride(npairs);
    c.yoff = y_offset(npairs);
    const int be = cblock_begin[grp + 1];
    int b0 = cblock_begin[grp];
    while (b0 < be && c.blocks[b0].level < level) ++b0;
    int b1 = b0;
    while (b1 < be && c.blocks[b1].level == level) ++b1;
    c.b0 = b0;
    c.b1 = b1;
    return c;
}

// Forward pass of one level (see combo_forward): the lane's product of the
// chord dx and its pending mark go to its column of the w_cprod planes.
__global__ void __launch_bounds__(256) combo_forward_kernel(run_args a, int level) {
    const int b = find_problem(a, offsetof(prob_desc, cb_block0), blockIdx.x);
    const prob_desc &d = descs(a)[b];
    const int64_t lane = ((int64_t)blockIdx.x - d.cb_block0) * blockDim.x + threadIdx.x;
    if (lane >= d.cb_lanes || level > d.levels) return;
    const combo_lane c = combo_lane_of(a, d, lane, level);
    if (c.b0 == c.b1) return;
    bool pending = false;
    const fe prod = combo_forward<false>(c.blocks, c.runs, c.b0, c.b1, c.tab, c.estride, pending);
    uint32_t *cp = at<uint32_t>(a, d.w_cprod) + lane;
#pragma unroll
    for (int w = 0; w < NL; ++w) cp[w * d.cb_lanes] = prod.v[w];
    cp[NL * d.cb_lanes] = pending ? 1u : 0u;
}

// Half of a level's lanes, in whole wavefronts: the backward pass runs one
// thread per two lanes, t and t + H.
__device__ __forceinline__ int64_t combo_half(int64_t lanes) { return ((lanes + 1) / 2 + 63) & ~(int64_t)63; }

// The combinations the chord formula does not cover (identity operands,
// x_a = x_b), marked by the passes: each finished on its own.
__device__ __forceinline__ void combo_rest(const combo_lane &c, bool pending) {
    for (int bi = c.b0; bi < c.b1; ++bi) {
        const plan_cblock blk = c.blocks[bi];
        for (int ri = blk.run_begin; ri < blk.run_end; ++ri) {
            const plan_crun run = c.runs[ri];
            for (int r = 0; r < CB; ++r) {
                if (run.dst[r] < 0) continue;
                uint32_t *slot = c.tab + run.dst[r] * c.estride;
                if (pending && (slot[NL - 1] & ENTRY_PENDING))
                    combo_special(c.tab + blk.a[r] * c.estride, c.tab + run.b * c.estride, c.yoff,
                                  (run.neg >> r) & 1, slot);
            }
        }
    }
}

// Backward pass of one level: a thread takes the lanes t and t + H, whose
// products share one inversion (1 / (p0 p1) times p1 and times p0), then the
// chord sums of each lane, and the rest.  A zero product (some chord of the
// lane has x_a = x_b) first sends the wavefront through the checked forward
// pass for that lane (its product is then nonzero) and later the matching
// checked backward pass; combinations the chord formula does not cover are
// finished in a third pass, which runs only when some lane of the wavefront
// has one.  With one thread per two lanes the kernel's wavefronts fill the
// chip in one round at two per SIMD, and half as many inversions run.
__global__ void __launch_bounds__(256) combo_backward_kernel(run_args a, int level) {
    const int b = find_problem(a, offsetof(prob_desc, cb_block0), blockIdx.x);
    const prob_desc &d = descs(a)[b];
    const int64_t t = ((int64_t)blockIdx.x - d.cb_block0) * blockDim.x + threadIdx.x;
    const int64_t H = combo_half(d.cb_lanes);
    if (t >= H || level > d.levels) return;  // whole wavefronts: H is a multiple of 64
    // (a lane's descriptor is looked up again in each loop rather than kept:
    // the backward pass needs nearly every register)
    auto lane_of = [&](int s, combo_lane &c) {
        const int64_t lane = t + s * H;
        if (lane >= d.cb_lanes) return false;
        c = combo_lane_of(a, d, lane, level);
        return c.b0 < c.b1;
    };
    bool pend0 = false, pend1 = false, safe0 = false, safe1 = false;
    fe prod0 = fe_one_mont(), prod1 = fe_one_mont();
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
        combo_lane c{};
        const bool live = lane_of(s, c);
        fe prod = fe_one_mont();
        bool pending = false;
        if (live) {
            const uint32_t *cp = at<const uint32_t>(a, d.w_cprod) + t + s * H;
#pragma unroll
            for (int w = 0; w < NL; ++w) prod.v[w] = cp[w * d.cb_lanes];
            pending = cp[NL * d.cb_lanes] != 0;
        }
        const bool safe = __ballot(live && fe_is_zero(prod)) != 0;
        if (safe && live) {
            pending = false;
            prod = combo_forward<true>(c.blocks, c.runs, c.b0, c.b1, c.tab, c.estride, pending);
        }
        if (s == 0) {
            pend0 = pending;
            safe0 = safe;
            prod0 = prod;
        } else {
            pend1 = pending;
            safe1 = safe;
            prod1 = prod;
        }
    }
    const fe inv = fe_inv(fe_mul_lq(prod0, prod1));
    const fe inv0 = fe_mul_lq(inv, prod1), inv1 = fe_mul_lq(inv, prod0);
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
        combo_lane c{};
        const bool live = lane_of(s, c);
        const bool pending = live && (s ? pend1 : pend0);
        const fe iv = fe_select(s != 0, inv0, inv1);
        if (s ? safe1 : safe0) {
            if (live) combo_backward<true>(c.blocks, c.runs, c.b0, c.b1, c.tab, c.estride, c.yoff, iv);
        } else if (live) {
            combo_backward<false>(c.blocks, c.runs, c.b0, c.b1, c.tab, c.estride, c.yoff, iv);
        }
        if (__ballot(pending)) combo_rest(c, pending);
    }
}

// --------------------------------------------------------------------------
// Accumulation (persistent)
// --------------------------------------------------------------------------
// Table entry of code word v (see pack_codes; nonzero) for pair p, read
// from global memory (the lanes of a wavefront share the pair, so they
// gather from one small table that L1 and L2 serve): x granule, then y
// granule, three loads each.  tp: the chunk's first table for the pair;
// est: bytes from one entry to the next (below 2^32).
__device__ __forceinline__ void load_entry(const uint32_t *tp, uint32_t est, int64_t yoff, int32_t v, u32x4 (&en)[4],
                                           uint32_t (&e8)[2]) {
    const uint32_t idx = (uint32_t)(v < 0 ? -v : v) - 1u;
    const uint32_t *ep = (const uint32_t *)((const char *)tp + (uint64_t)idx * est);
    en[0] = *(const u32x4 *)ep;
    en[1] = *(const u32x4 *)(ep + 4);
    e8[0] = ep[8];
    en[2] = *(const u32x4 *)(ep + yoff);
    en[3] = *(const u32x4 *)(ep + yoff + 4);
    e8[1] = ep[yoff + 8];
}

// One tile: rows bx * tm .. + tm, (j, point) pairs by * pp .. + pp, column
// groups of split bz.  Each lane walks its row's nonzero codes and adds the
// entries T[k][j, pt][|code|] (negated for negative codes) into its
// accumulator; entries come straight from the tables in global memory, so
// one code list per split covers all of the split's groups and a wavefront
// runs as many additions as its rows' largest count of nonzero codes.
__device__ __forceinline__ void accumulate_tile(const run_args &a, const prob_desc &d, int bx, int by, int bz) {
    const int tid = threadIdx.x;
    const int tm = d.tm, emax = d.emax, m = d.m, l = d.l;
    const int row_l = tid % tm;
    const int pair_l = tid / tm;
    const int i = bx * tm + row_l;
    const int p = by * d.pp + pair_l;
    const int npairs = 2 * l;
    if (i >= m || p >= npairs) return;
    const int g_begin = bz * d.gps;
    const int g_end = min(d.ngroups, g_begin + d.gps);
    const uint32_t *table = at<const uint32_t>(a, d.w_table);
    const int32_t *lists = plan_at<int32_t>(a, d.o_lists);
    const int64_t *chunk_off = plan_at<int64_t>(a, d.o_chunk_off);
    const int32_t *chunk_len = plan_at<int32_t>(a, d.o_chunk_len);
    const uint32_t est = (uint32_t)(entry_stride(npairs) * 4);  // bytes from one entry to the next
    const int64_t yoff = y_offset(npairs);

    // the accumulator in XYZZ coordinates (ec.hpp), converted to Jacobian
    // once, at the store
    xpt acc = xpt_infinity();
    bool acc_inf = true;  // whether acc is the identity, kept by the additions
    for (int gc = g_begin; gc < g_end; gc += d.kc) {
        const int chunk = bz * d.chunks_per_split + (gc - g_begin) / d.kc;
        const int len = chunk_len[chunk];
        const int32_t *lst = lists + chunk_off[chunk] * m + i;
        const uint32_t *tp = entry_at((uint32_t *)table, npairs, emax, gc, 0, p);
        // software pipeline: codes three slots ahead, the entry one slot
        // ahead, so that their memory latency overlaps the point additions
        int32_t v_cur = len > 0 ? lst[0] : 0;
        int32_t v_nxt = len > 1 ? lst[m] : 0;
        int32_t v_nx2 = len > 2 ? lst[2 * (int64_t)m] : 0;
        u32x4 en[4];
        uint32_t e8[2];
        if (v_cur != 0) {
            load_entry(tp, est, yoff, v_cur, en, e8);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) en[q] = u32x4{0u, 0u, 0u, 0u};
            e8[0] = e8[1] = 0u;
        }
        for (int it = 0; it < len; ++it) {
            const int32_t v = v_cur;
            const u32x4 ec[4] = {en[0], en[1], en[2], en[3]};
            const uint32_t c8[2] = {e8[0], e8[1]};
            v_cur = v_nxt;
            v_nxt = v_nx2;
            if (it + 3 < len) v_nx2 = lst[(int64_t)(it + 3) * m];
            if (it + 1 < len && v_cur != 0) load_entry(tp, est, yoff, v_cur, en, e8);
            if (v == 0) continue;  // padding after the row's last nonzero code
            apt Q = {{{ec[0].x, ec[0].y, ec[0].z, ec[0].w, ec[1].x, ec[1].y, ec[1].z, ec[1].w, c8[0] & LIMB8_BITS}},
                     {{ec[2].x, ec[2].y, ec[2].z, ec[2].w, ec[3].x, ec[3].y, ec[3].z, ec[3].w, c8[1]}}};
            // an identity entry leaves the sum as it is: the lane skips it,
            // so the addition never reads the old accumulator after its
            // formulas (the result can take its registers)
            if (c8[0] & ENTRY_INF) continue;
            if (v < 0) Q.y = fe_neg(Q.y);
            acc = xpt_add_affine_known(acc, acc_inf, Q, false, acc_inf);
        }
    }
    const int j = p >> 1, pt = p & 1;
    const int64_t e_out = (int64_t)i * l + j;
    if (d.direct) {
        // the row's only entry was added to the identity, so acc = (x, y, 1,
        // 1) or the identity: already affine
        apt A;
        A.x = acc_inf ? fe_zero() : acc.X;
        A.y = acc_inf ? fe_zero() : acc.Y;
        store_affine(a.io[d.io].C, a.io[d.io].ldc, pt, e_out, A);
        return;
    }
    const jpt J = xpt_to_jpt(acc, acc_inf);
    if (d.S > 1) {
        store_jac_m(at<uint32_t>(a, d.w_part) + (int64_t)bz * JAC2_PLANES * d.ldj, d.ldj, pt, e_out, J);
    } else if (d.c_form == PCMM_AFFINE) {
        store_jac_m(at<uint32_t>(a, d.w_cjac), d.ldj, pt, e_out, J);
    } else {
        store_jac(a.io[d.io].C, a.io[d.io].ldc, pt, e_out, J);
    }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) accumulate_kernel(run_args a) {
    __shared__ int32_t s_tile;
    int32_t *ctr = at<int32_t>(a, a.ctr_off);
    for (;;) {
        __syncthreads();  // every thread has read s_tile
        if (threadIdx.x == 0) s_tile = atomicAdd(ctr, 1);
        __syncthreads();
        const int64_t tile = __builtin_amdgcn_readfirstlane(s_tile);  // uniform over the workgroup
        if (tile >= a.total_tiles) return;
        const int b = find_problem(a, offsetof(prob_desc, tile0), tile);
        const prob_desc &d = descs(a)[b];
        const int64_t u = tile - d.tile0;
        const int64_t txy = (int64_t)d.tiles_x * d.tiles_y;
        const int bz = (int)(u / txy);
        const int64_t r = u - (int64_t)bz * txy;
        const int by = (int)(r / d.tiles_x);
        const int bx = (int)(r - (int64_t)by * d.tiles_x);
        accumulate_tile(a, d, bx, by, bz);
    }
}

// Sum of the S (power of two <= 64) split-k partial sums of each output
// point.  An output's partials are spread over RL = min(S, 8) consecutive
// lanes; lane q adds partials q, q + RL, ... sequentially (every addition is
// useful), then the RL lanes combine by a shuffle tree of log2(RL) levels.
// A problem's threads start at a block boundary and RL divides 64, so the
// lanes of one output are in one wavefront.
constexpr int REDUCE_LANES = 8;

__global__ void __launch_bounds__(256) reduce_kernel(run_args a) {
    const int b = find_problem(a, offsetof(prob_desc, red_block0), blockIdx.x);
    const prob_desc &d = descs(a)[b];
    const int64_t t = ((int64_t)blockIdx.x - d.red_block0) * blockDim.x + threadIdx.x;
    const int S = d.S;
    const int RL = S < REDUCE_LANES ? S : REDUCE_LANES;
    const int64_t n_out = (int64_t)d.m * d.l;
    const int q = (int)(t % RL);
    const int64_t rest = t / RL;  // (e, pt) pairs, pt fastest
    const bool valid = rest < 2 * n_out;
    const int64_t e = valid ? rest >> 1 : 0;
    const int pt = (int)(rest & 1);
    const uint32_t *part = at<const uint32_t>(a, d.w_part);
    jpt P = jpt_infinity();
    if (valid) {
        P = load_jac_m(part + (int64_t)q * JAC2_PLANES * d.ldj, d.ldj, pt, e);
        for (int s = q + RL; s < S; s += RL)
            P = jpt_add(P, load_jac_m(part + (int64_t)s * JAC2_PLANES * d.ldj, d.ldj, pt, e));
    }
    for (int off = RL >> 1; off >= 1; off >>= 1) {
        jpt Q;
#pragma unroll
        for (int w = 0; w < NL; ++w) {
            Q.X.v[w] = __shfl_down(P.X.v[w], off, 64);
            Q.Y.v[w] = __shfl_down(P.Y.v[w], off, 64);
            Q.Z.v[w] = __shfl_down(P.Z.v[w], off, 64);
        }
        jpt R = jpt_add(P, Q);
        if (q < off) P = R;
    }
    if (valid && q == 0) {
        if (d.c_form == PCMM_AFFINE) store_jac_m(at<uint32_t>(a, d.w_cjac), d.ldj, pt, e, P);
        else store_jac(a.io[d.io].C, a.io[d.io].ldc, pt, e, P);
    }
}

__global__ void __launch_bounds__(256) normalize_batch_kernel(run_args a) {
    const int b = find_problem(a, offsetof(prob_desc, norm_block0), blockIdx.x);
    const prob_desc &d = descs(a)[b];
    const int64_t t = ((int64_t)blockIdx.x - d.norm_block0) * blockDim.x + threadIdx.x;
    normalize_points<true, false>(at<const uint32_t>(a, d.w_cjac), d.ldj, a.io[d.io].C, a.io[d.io].ldc,
                                  (int64_t)d.m * d.l, 2, at<uint32_t>(a, d.w_norm), d.ld_pre, d.norm_per, t,
                                  d.norm_threads);
}

__global__ void fill_infinity_kernel(uint32_t *out, int64_t ld, int64_t n, int form) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    for (int pt = 0; pt < 2; ++pt)
        for (int c = 0; c < form; ++c)
            for (int w = 0; w < 8; ++w) out[((int64_t)(pt * form + c) * 8 + w) * ld + e] = 0u;
}

// --------------------------------------------------------------------------
// Host side: configuration, autotuning, geometry
// --------------------------------------------------------------------------
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool valid_cfg(const pcmm_cussen_cfg *cfg) {
    if (!cfg) return true;
    if (cfg->rounds < 0 || cfg->rounds > 8 || cfg->group < PCMM_GROUP_AUTO || cfg->group > 4 ||
        cfg->k_split < 0 || cfg->k_split > 64 || cfg->k_chunk < 0 || cfg->profile < 0)
        return false;
    if (cfg->k_split > 0 && (cfg->k_split & (cfg->k_split - 1))) return false;
    return true;
}

int cfg_rounds(const pcmm_cussen_cfg *cfg) { return cfg && cfg->rounds > 0 ? cfg->rounds : 4; }

// Accumulation tile: rows per tile, the fewest padded rows, the larger tile
// on ties (the wavefronts of a workgroup then gather from the same pairs'
// tables); pp (j, point) pairs per tile of 256 lanes.
struct acc_tiling {
    int tm, pp, tiles_x, tiles_y;
};

acc_tiling acc_tiles(int m, int l) {
    acc_tiling t;
    t.tm = 256;
    for (int tm : {128, 64, 32})
        if ((int64_t)(m + tm - 1) / tm * tm < (int64_t)(m + t.tm - 1) / t.tm * t.tm) t.tm = tm;
    t.pp = 256 / t.tm;
    t.tiles_x = (m + t.tm - 1) / t.tm;
    t.tiles_y = (2 * l + t.pp - 1) / t.pp;
    return t;
}

// The autotuner's cost model: predicted GPU milliseconds of the parts of a
// run that depend on the column group g and the split S of the inner
// dimension (the digit tables are the same for every g and S), fitted to
// kernel times measured on MI355X at 17 shapes (512^3 and 128^3 at 1..8
// bits, the serving layer 256 x 1024 x 8 with S = 1..64, a sample of the
// uneven batch; g = 1..4); it picks the measured best g for 16 of them and
// the 17th within 4 %.
//   accumulation  persistent: a tile's time is its rows' chain of mixed
//                 additions (nonzero codes per row and split) times tau;
//                 tiles run W = 512 at a time (2 per CU, as when the model
//                 was fitted; the kernel now keeps 3 per CU at about the
//                 same throughput), and a tile alone still takes beta of
//                 its time under full load
//   combinations  throughput (all combinations) or, with few lanes, one
//                 lane's chain: an inversion per level and its share of the
//                 group's combinations; 2048 wavefronts resident
//   reduction     (S > 1) per output, min(S, 8) lanes adding S / min(S, 8)
//                 partials each, then a shuffle tree
double predicted_ms(const cussen_plan &P, int l, int S) {
    constexpr double TAU = 8.35e-3, BETA = 0.618, ACC0 = 0.043;
    constexpr double COMBO = 1.361e-7, COMBO_LANE = 8.79e-3, COMBO_LEVEL = 5.77e-2, COMBO0 = 0.0382;
    constexpr double RED0 = 0.0322, RED = 0.0936e-6;
    constexpr double W = 512, WAVES = 2048;
    const int m = std::max(P.m, 1);
    const acc_tiling t = acc_tiles(m, l);
    const double tiles = (double)t.tiles_x * t.tiles_y * S;
    const double pairs = 2.0 * l;
    double ms = ACC0 + TAU * ((double)P.accum_adds / m / S) * std::max(tiles / W, BETA);
    if (!P.combos.empty()) {
        const double rounds = std::max(1.0, std::ceil((double)P.ngroups * pairs / 64 / WAVES));
        const double lane = COMBO_LEVEL * (std::min(P.g, P.n) - 1) + COMBO_LANE * (double)P.combo_adds / P.ngroups;
        ms += COMBO0 + std::max(COMBO * (double)P.combo_adds * pairs, lane * rounds);
    }
    if (S > 1) {
        const double s8 = std::min(S, 8);
        ms += RED0 + RED * P.m * pairs * s8 * ((double)S / s8 + std::log2(s8));
    }
    return ms;
}

// Splits of the inner dimension the tuner considers: powers of two up to 64,
// each split holding at least two column groups.
int max_split(const cussen_plan &P) {
    int S = 1;
    while (S < 64 && P.ngroups / (S * 2) >= 2) S *= 2;
    return S;
}

// (m, n, l, bits, signed, N, requested group, requested split) -> (g, S)
using tune_key = std::tuple<int, int, int, int, int, int, int, int>;
std::mutex g_tune_lock;
std::map<tune_key, std::pair<int, int>> g_tune_cache;

// host threads for planning: the CPU share of one GPU
int host_threads() { return std::max(1, std::min(16, (int)std::thread::hardware_concurrency())); }

// Builds the plan for cfg's group, or for the autotuned one, and picks the
// split of the inner dimension (cfg's, else the model's best), on up to
// `threads` host threads.  l: output columns the plan runs with.
int build_plan_cfg(const void *A, int m, int n, int l, int bits, bool sgn, const pcmm_cussen_cfg *cfg,
                   cussen_plan *out, int *split, int threads) {
    const int N = cfg_rounds(cfg);
    const int group = cfg ? cfg->group : 0;
    const int req_split = cfg && cfg->k_split > 0 ? cfg->k_split : 0;
    auto over_cap = [](const cussen_plan &P) {
        return P.g > 1 && (size_t)std::max(P.max_entries, 1) * ENTRY_WORDS * 4 > GROUP_TABLE_CAP;
    };
    // the best split of one plan under the model
    auto best_split = [&](const cussen_plan &P, double *cost) {
        int bs = req_split ? req_split : 1;
        double bc = predicted_ms(P, l, bs);
        if (!req_split)
            for (int S = 2; S <= max_split(P); S *= 2) {
                const double c = predicted_ms(P, l, S);
                if (c < bc) {
                    bc = c;
                    bs = S;
                }
            }
        if (cost) *cost = bc;
        return bs;
    };
    if (group != PCMM_GROUP_AUTO) {
        int rc = build_cussen_plan(A, m, n, bits, sgn, N, group > 0 ? group : 1, out, threads);
        if (!rc) *split = best_split(*out, nullptr);
        return rc;
    }
    const tune_key key{m, n, l, bits, (int)sgn, N, group, req_split};
    std::pair<int, int> cached{0, 0};
    {
        std::lock_guard<std::mutex> guard(g_tune_lock);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) cached = it->second;
    }
    if (cached.first > 0) {
        // the choice was made on another matrix of the same shape: its group
        // tables are re-checked against the cap on this one
        int rc = build_cussen_plan(A, m, n, bits, sgn, N, cached.first, out, threads);
        if (!rc && !over_cap(*out)) {
            *split = cached.second;
            return 0;
        }
        if (rc && cached.first == 1) return rc;
        rc = build_cussen_plan(A, m, n, bits, sgn, N, 1, out, threads);
        if (!rc) *split = best_split(*out, nullptr);
        return rc;
    }
    int best_g = 1, best_s = 1;
    double best = 0;
    // a code keys g digits of 9 bits (entries up to 8 bits) or 17 bits (9..16
    // bits) into 64 bits, so wide entries allow at most 3 columns per group
    const int gmax = std::max(1, std::min(bits <= 8 ? 4 : 3, n));
    for (int g = 1; g <= gmax; ++g) {
        cussen_plan P;
        int rc = build_cussen_plan(A, m, n, bits, sgn, N, g, &P, threads);
        if (rc && g == 1) return rc;
        if (rc || over_cap(P)) continue;  // a group too large for the plan's limits is no candidate
        double c;
        const int S = best_split(P, &c);
        if (g == 1 || c < best) {
            best = c;
            best_g = g;
            best_s = S;
            *out = std::move(P);
        }
    }
    *split = best_s;
    std::lock_guard<std::mutex> guard(g_tune_lock);
    g_tune_cache[key] = {best_g, best_s};
    return 0;
}

// Per-problem geometry and the sizes of its workspace regions.
struct job {
    cussen_plan P;
    int index = 0;  // the caller's problem index (matrices of the run)
    int l = 0, c_form = PCMM_AFFINE;
    int J = 1, Lj = 1;
    int64_t n_lanes = 0;
    int64_t cb_lanes = 0;     // combination lanes: (group, pair), if the plan has combinations
    int Lj_pad = 0;           // table-build lanes with each unit padded to a
    int64_t n_lanes_pad = 0;  // whole wavefront (0: not applicable), chosen per run
    size_t regs_bytes_pad = 0;
    int coop_w = 0;           // padded runs: lanes sharing each level-1 chain (0: none)
    int coop_lpu = 0;         // lanes per unit in the cooperative build (whole wavefronts)
    int coop_h = 0;           // register slots of the ops before the level-1 chain
    int coop_slots = 0;       // register slots per lane: coop_h + the largest block
    int64_t n_lanes_coop = 0;
    size_t regs_bytes_coop = 0;
    int tm = 256, pp = 1, kc = 1, S = 1, gps = 0, tiles_x = 1, tiles_y = 1;
    int64_t ldj = 64, norm_threads = 0, ld_pre = 0;
    int norm_per = 0;
    bool direct = false;  // see prob_desc::direct
    size_t regs_bytes = 0, table_bytes = 0, part_bytes = 0, cjac_bytes = 0, norm_bytes = 0, cprod_bytes = 0;
    size_t footprint = 0;  // workspace bytes of this problem's regions
    double tile_cost = 0;
    int chunks_per_split = 0;
    std::vector<int32_t> lists, chunk_len;
    std::vector<int64_t> chunk_off;
};

// padded table-build lanes allowed (4 wavefronts per SIMD of a 256-CU device)
constexpr int64_t PAD_LANES_MAX = 4 * 1024 * 64;

// whether a run pads its groups' table-build lanes: only if the padded grid
// of all its problems stays within PAD_LANES_MAX
template <typename JobOf>
bool pad_run(size_t count, JobOf job_at) {
    int64_t lanes = 0;
    for (size_t q = 0; q < count; ++q) {
        const auto &G = job_at(q);
        lanes += G.coop_w > 1 ? G.n_lanes_coop : G.n_lanes_pad ? G.n_lanes_pad : G.n_lanes;
    }
    return lanes <= PAD_LANES_MAX;
}

// Whether every unit (column) ends its program with its level-1
// reconstruction, the prefix sums S_i = S_{i-1} + b_i (S_0 = b_0, the digit
// table's entry 0): then lanes of a padded unit can share that chain.
bool level1_chains(const cussen_plan &P) {
    for (int u = 0; u < P.nunits; ++u) {
        const int eb = P.entry_begin[u], E = P.entry_begin[u + 1] - eb;
        const int ob = P.op_begin[u], oe = P.op_begin[u + 1];
        if (E == 0) continue;  // an all-zero column: no table
        if (oe - ob < E - 1) return false;
        for (int i = 1; i < E; ++i) {
            const plan_op &op = P.ops[oe - (E - 1) + (i - 1)];
            if (op.kind != OP_ADD || op.neg_b || op.a != P.entries[eb + i - 1] || op.dst != P.entries[eb + i])
                return false;
        }
    }
    return true;
}

void make_geometry(job &G, const pcmm_cussen_cfg *cfg, int split) {
    const cussen_plan &P = G.P;
    const int m = P.m, l = G.l;
    const int emax = std::max(P.max_entries, 1);
    // digit tables: J chains per lane so that one inversion serves >= ~64
    // entries, while keeping >= ~16K lanes
    double avg_e = P.nunits ? (double)P.digit_entries / P.nunits : 1.0;
    int J = 1;
    while (J < 8 && 2.0 * J * std::max(avg_e, 1.0) <= 64.0) J *= 2;
    while (J > 1 && (int64_t)P.nunits * 2 * ((l + J - 1) / J) < 16384) J /= 2;
    G.J = J;
    G.Lj = (l + J - 1) / J;
    // lanes of one unit fill whole wavefronts (uniform control flow) when
    // possible.  With few output columns a unit's chains fill less than a
    // wavefront; packing several units into one wavefront runs their
    // different programs divergently, so a run pads each unit to a whole
    // wavefront when its padded grid stays small (pad_run): the build is then
    // bound by its chains' latency, not by lanes.
    if (2 * G.Lj >= 64) G.Lj = (G.Lj + 31) / 32 * 32;
    else G.Lj_pad = 32;
    G.n_lanes = (int64_t)P.nunits * 2 * G.Lj;
    G.n_lanes_pad = G.Lj_pad ? (int64_t)P.nunits * 2 * G.Lj_pad : 0;
    G.cb_lanes = P.combos.empty() ? 0 : (int64_t)P.ngroups * 2 * l;
    // a padded unit has 64 lanes for its 2 l chains: up to W = 64 / (2 l)
    // lanes (a power of two) split each level-1 chain as a parallel scan
    // instead of idling, with W chosen by the chain's depth
    G.coop_w = 0;
    if (G.Lj_pad && l >= 1 && level1_chains(P)) {
        // A lane's work in mixed additions: its chain (E - 1 alone; with W
        // lanes per chain a ladder to its block's start, a doubling and an
        // addition per bit of the largest value, then E / W - 1 additions),
        // the inversion (~25) and the conversions (~0.5 each).  A wavefront
        // alone on its SIMD issues at about half rate (dependent products),
        // so the time is the larger of twice a wavefront's work and the
        // wavefronts per SIMD times it (1024 SIMDs of 64 lanes).
        int32_t vmax = 1;
        for (int32_t v : P.entry_value) vmax = std::max(vmax, v);
        const double vbits = 32 - __builtin_clz((uint32_t)vmax);
        auto lpu = [&](int W) { return ((int64_t)2 * l * W + 63) / 64 * 64; };
        auto cost = [&](int W) {
            const double bs = W == 1 ? avg_e : std::ceil(avg_e / W);
            const double chain = W == 1 ? std::max(avg_e - 1.0, 0.0) : 2.0 * (vbits - 1.0) + bs - 1.0;
            const double work = chain + 25.0 + 0.5 * bs;
            const double waves = std::ceil((double)P.nunits * (W == 1 ? 64 : lpu(W)) / 65536.0);
            return std::max(2.0, waves) * work;
        };
        int best = 1;
        for (int W = 2; W <= 64 && (int64_t)P.nunits * lpu(W) <= PAD_LANES_MAX; W *= 2)
            if (cost(W) < cost(best)) best = W;
        if (best >= 2) {
            G.coop_w = best;
            G.coop_lpu = (int)lpu(best);
            // registers of the ops before each chain keep their numbers; a
            // lane's block of chain entries follows them
            int h = 0, emax_u = 0;
            for (int u = 0; u < P.nunits; ++u) {
                const int E = P.entry_begin[u + 1] - P.entry_begin[u];
                emax_u = std::max(emax_u, E);
                const int ofirst = P.op_begin[u + 1] - std::max(E - 1, 0);
                for (int o = P.op_begin[u]; o < ofirst; ++o) h = std::max(h, P.ops[o].dst + 1);
                if (E > 0 && P.entries[P.entry_begin[u]] >= 0) h = std::max(h, P.entries[P.entry_begin[u]] + 1);
            }
            G.coop_h = h;
            G.coop_slots = std::max(1, h + (emax_u + best - 1) / best);
            G.n_lanes_coop = (int64_t)P.nunits * G.coop_lpu;
            G.regs_bytes_coop = (size_t)G.coop_slots * JAC_WORDS * 4 * (size_t)G.n_lanes_coop;
        }
    }
    // accumulation tile and the split of the inner dimension
    const int npairs = 2 * l;
    const acc_tiling t = acc_tiles(m, l);
    G.tm = t.tm;
    G.pp = t.pp;
    G.tiles_x = t.tiles_x;
    G.tiles_y = t.tiles_y;
    int S = std::max(split, 1);
    while (S > 1 && (P.ngroups + S - 1) / S < 1) S /= 2;
    G.S = S;
    G.gps = P.ngroups > 0 ? (P.ngroups + S - 1) / S : 0;
    // column groups per code list: a split's groups in one list, unless the
    // caller asks for shorter lists (each list is padded to its longest row);
    // a code word is a signed entry index over the list's groups' tables, so
    // a list covers fewer than 2^31 / E groups
    const int max_list_groups = (int)std::min<int64_t>(INT32_MAX - 1, (INT32_MAX - 1) / std::max(P.max_entries, 1));
    G.kc = std::max(1, std::min({cfg && cfg->k_chunk > 0 ? cfg->k_chunk : G.gps, std::max(G.gps, 1),
                                 max_list_groups}));
    G.tile_cost = (double)G.tm * G.pp * G.gps;
    // workspace regions
    const int64_t n_out = (int64_t)m * l;
    G.ldj = std::max<int64_t>(64, (n_out + 63) / 64 * 64);
    G.regs_bytes = (size_t)G.J * std::max(P.max_regs, 1) * JAC_WORDS * 4 * (size_t)G.n_lanes;
    G.regs_bytes_pad = (size_t)G.J * std::max(P.max_regs, 1) * JAC_WORDS * 4 * (size_t)G.n_lanes_pad;
    G.table_bytes = (size_t)P.ngroups * npairs * emax * ENTRY_WORDS * 4;
    G.part_bytes = S > 1 ? (size_t)S * JAC2_PLANES * G.ldj * 4 : 0;
    const bool affine = G.c_form == PCMM_AFFINE;
    // one column group and one split: a row's output is its single table
    // entry (affine already, or the identity), written without normalisation
    G.direct = affine && P.ngroups <= 1 && S == 1;
    G.cjac_bytes = affine && !G.direct ? (size_t)JAC2_PLANES * G.ldj * 4 : 0;
    G.norm_threads = G.norm_per = 0;
    G.ld_pre = 0;
    G.norm_bytes = 0;
    if (affine && !G.direct) {
        normalize_geometry(n_out, &G.norm_threads, &G.norm_per);
        G.ld_pre = G.norm_threads * G.norm_per * 2;
        G.norm_bytes = normalize_scratch_bytes(n_out, 2);
    }
    // (a padded run uses the cooperative register file when there is one)
    G.cprod_bytes = (size_t)G.cb_lanes * (NL + 1) * 4;
    G.footprint = align256(std::max(G.regs_bytes, G.coop_w > 1 ? G.regs_bytes_coop : G.regs_bytes_pad)) +
                  align256(G.table_bytes) +
                  align256(G.part_bytes) +
                  align256(G.cjac_bytes) + align256(G.norm_bytes) + align256(G.cprod_bytes);
}

// The accumulation walks, per (split, chunk of kc column groups), only the
// nonzero codes of each row: slot-major lists lists[(chunk_off + slot) * m
// + i] = +-(q E + e + 1) for code +-(e + 1) of the chunk's group q (E: the
// table stride in entries), i.e. the entry's index over the chunk's tables
// with the code's sign, padded with 0 (no operation) up to the chunk's
// longest row.  A wavefront then runs as many
// mixed additions as its rows' largest count of nonzero codes rather than
// one per column group, which matters where many codes are zero (small
// bit-widths).
void pack_codes(job &G, int threads) {
    const cussen_plan &P = G.P;
    const int m = P.m;
    const int32_t E = std::max(P.max_entries, 1);  // the kernels' emax
    G.chunks_per_split = G.gps > 0 ? (G.gps + G.kc - 1) / G.kc : 0;
    const int nchunks = G.S * G.chunks_per_split;
    G.chunk_off.assign(nchunks, 0);
    G.chunk_len.assign(nchunks, 0);
    auto chunk_groups = [&](int c, int &g0, int &g1) {
        const int bz = c / std::max(G.chunks_per_split, 1);
        g0 = bz * G.gps + (c % std::max(G.chunks_per_split, 1)) * G.kc;
        g1 = std::min({P.ngroups, bz * G.gps + G.gps, g0 + G.kc});
    };
    // rows are independent (each owns one column of every list): ranges of
    // rows on up to `threads` threads, first for the lists' lengths, then to
    // fill them
    // (a thread costs tens of microseconds to start: each gets >= 64 K codes)
    const int nthreads =
        (int)std::max<int64_t>(1, std::min<int64_t>({threads, m / 64, (int64_t)m * P.ngroups / 65536}));
    auto run = [&](auto &&body) {
        if (nthreads <= 1) {
            body(0, m, 0);
            return;
        }
        std::vector<std::thread> pool;
        for (int t = 0; t < nthreads; ++t)
            pool.emplace_back(body, (int)((int64_t)m * t / nthreads), (int)((int64_t)m * (t + 1) / nthreads), t);
        for (auto &th : pool) th.join();
    };
    std::vector<int> part_len((size_t)nthreads * std::max(nchunks, 1), 0);
    run([&](int r0, int r1, int t) {
        for (int c = 0; c < nchunks; ++c) {
            int g0, g1, len = 0;
            chunk_groups(c, g0, g1);
            for (int i = r0; i < r1; ++i) {
                int k = 0;
                for (int g = g0; g < g1; ++g) k += P.codes[(size_t)g * m + i] != 0;
                len = std::max(len, k);
            }
            part_len[(size_t)t * nchunks + c] = len;
        }
    });
    int64_t total = 0;
    for (int c = 0; c < nchunks; ++c) {
        int len = 0;
        for (int t = 0; t < nthreads; ++t) len = std::max(len, part_len[(size_t)t * nchunks + c]);
        G.chunk_off[c] = total;
        G.chunk_len[c] = len;
        total += len;
    }
    G.lists.assign((size_t)total * m, 0);
    run([&](int r0, int r1, int) {
        std::vector<int32_t> cnt(std::max(r1 - r0, 0));
        for (int c = 0; c < nchunks; ++c) {
            int g0, g1;
            chunk_groups(c, g0, g1);
            std::fill(cnt.begin(), cnt.end(), 0);
            for (int g = g0; g < g1; ++g) {
                const int16_t *row = &P.codes[(size_t)g * m];
                for (int i = r0; i < r1; ++i) {
                    if (!row[i]) continue;
                    const int32_t idx = (int32_t)(g - g0) * E + std::abs((int)row[i]);
                    G.lists[(size_t)(G.chunk_off[c] + cnt[i - r0]++) * m + i] = row[i] < 0 ? -idx : idx;
                }
            }
        }
    });
}

}  // namespace

namespace {

// One phase of a run: a subset of its problems, queued as table build,
// combinations, persistent accumulation, reduction and normalisation; the
// phases of a run reuse one workspace region one after another.
struct run_phase {
    int32_t count = 0;    // descriptors
    size_t desc_off = 0;  // byte offset of the phase's descriptors in the workspace
    int64_t tb_blocks = 0, cb_blocks = 0, tiles = 0, red_blocks = 0, norm_blocks = 0;
    int acc_grid = 0;
    int levels = 1;       // largest combination level of the phase's problems (1: none)
    bool coop = false;    // some problem's tables are built by coop_table_kernel
};

// What a run queues: the image (descriptor blocks, plan arrays) copied to the
// start of the workspace, the accumulation queue counter after it, then the
// problems' regions.
struct run_layout {
    std::vector<run_phase> phases;  // empty: no GPU work
    size_t copy_bytes = 0, ctr_off = 0, ws_bytes = 256;
    std::vector<int> fills;  // run indices whose inner dimension is empty (identity outputs)
};

// A run whose problems together need more workspace than this is split into
// phases (first fit by decreasing footprint); a problem larger than the
// limit is a phase of its own.
constexpr size_t PHASE_WORKSPACE_LIMIT = (size_t)14000000000ull;

// pinned staging for descriptor blocks of selected runs; an event guards reuse
struct stage_slot {
    void *host = nullptr;
    hipEvent_t done = nullptr;
};

}  // namespace

// A compiled set of problems (the executor's unit; pcmm_cussen builds one of
// a single problem per call).
struct pcmm_plan_s {
    int device = 0;
    int count = 0;
    std::vector<int32_t> m, n, l, c_form;
    std::vector<pcmm_cussen_stats> stats;
    std::vector<job> jobs;     // problems with GPU work, in execution order
    std::vector<int> job_of;   // problem index -> job index, or -1
    std::vector<prob_desc> desc;  // the full run's descriptors (templates of selected runs)
    std::vector<char> image;   // descriptors + plan arrays
    void *pinned = nullptr;    // immutable pinned copy of `image` (plans only)
    run_layout full;           // the run of every problem once
    const char *resident = nullptr;  // device copy of the image (pcmm_plan_make_resident)
    std::mutex stage_lock;
    std::vector<stage_slot> ring;
    int ring_next = 0;
    ~pcmm_plan_s() {
        if (pinned) (void)hipHostFree(pinned);  // destructors report nothing
        for (auto &r : ring) {
            if (r.host) (void)hipHostFree(r.host);
            if (r.done) (void)hipEventDestroy(r.done);
        }
    }
};

namespace {

void fill_stats(const job &G, pcmm_cussen_stats *st) {
    memset(st, 0, sizeof *st);
    const cussen_plan &P = G.P;
    st->level_mults = P.level_mults;
    st->level_adds = P.level_adds;
    st->table_entries = P.table_entries;
    st->table_adds = P.table_adds;
    st->accum_adds = P.accum_adds;
    st->max_entries = P.max_entries;
    st->workspace_bytes = (int64_t)G.footprint;
    st->k_split = G.S;
    st->lanes_per_chain = G.J;
    st->group = P.g;
    st->combo_adds = P.combo_adds;
    st->digit_entries = P.digit_entries;
}

// Lays out descriptors, plan image and workspace regions of the plan's jobs,
// and sizes the grids of the non-persistent kernels.  Jobs are packed into
// phases of at most PHASE_WORKSPACE_LIMIT bytes of regions each (first fit,
// largest footprint first); within a phase the most expensive accumulation
// tiles come first (the queue hands them out in order).
pcmm_status finish_plan(pcmm_plan_s &pl) {
    const size_t nd = pl.jobs.size();
    std::vector<size_t> phase_of(nd, 0);
    size_t nphases = nd ? 1 : 0;
    {
        size_t total = 0;
        for (const job &G : pl.jobs) total += G.footprint;
        if (total > PHASE_WORKSPACE_LIMIT) {
            std::vector<size_t> idx(nd);
            for (size_t k = 0; k < nd; ++k) idx[k] = k;
            std::stable_sort(idx.begin(), idx.end(),
                             [&](size_t x, size_t y) { return pl.jobs[x].footprint > pl.jobs[y].footprint; });
            std::vector<size_t> used;
            for (size_t k : idx) {
                size_t p = 0;
                while (p < used.size() && used[p] + pl.jobs[k].footprint > PHASE_WORKSPACE_LIMIT) ++p;
                if (p == used.size()) used.push_back(0);
                used[p] += pl.jobs[k].footprint;
                phase_of[k] = p;
            }
            nphases = used.size();
        }
    }
    // execution order: by phase, then most expensive accumulation tiles first
    {
        std::vector<size_t> order(nd);
        for (size_t k = 0; k < nd; ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
            if (phase_of[x] != phase_of[y]) return phase_of[x] < phase_of[y];
            return pl.jobs[x].tile_cost > pl.jobs[y].tile_cost;
        });
        std::vector<job> jobs;
        std::vector<size_t> ph;
        jobs.reserve(nd);
        for (size_t k : order) {
            jobs.push_back(std::move(pl.jobs[k]));
            ph.push_back(phase_of[k]);
        }
        pl.jobs = std::move(jobs);
        phase_of = std::move(ph);
    }
    run_layout &L = pl.full;
    L.phases.assign(nphases, run_phase{});
    size_t img = 0;
    for (size_t p = 0; p < nphases; ++p) {
        size_t cnt = 0;
        for (size_t k = 0; k < nd; ++k) cnt += phase_of[k] == p;
        L.phases[p].count = (int32_t)cnt;
        L.phases[p].desc_off = img;
        img += align256(cnt * sizeof(prob_desc));
    }
    std::vector<prob_desc> D(nd);
    for (size_t k = 0; k < nd; ++k) {
        const job &G = pl.jobs[k];
        D[k] = prob_desc{};
        auto arr = [&](int64_t &off, size_t bytes) {
            off = (int64_t)img;
            img += align256(bytes);
        };
        arr(D[k].o_ops, G.P.ops.size() * sizeof(plan_op));
        arr(D[k].o_unit_col, G.P.unit_col.size() * 4);
        arr(D[k].o_unit_grp, G.P.unit_grp.size() * 4);
        arr(D[k].o_unit_off, G.P.unit_off.size() * 4);
        arr(D[k].o_cblock_begin, G.P.cblock_begin.size() * 4);
        arr(D[k].o_cblocks, G.P.cblocks.size() * sizeof(plan_cblock));
        arr(D[k].o_cruns, G.P.cruns.size() * sizeof(plan_crun));
        arr(D[k].o_op_begin, G.P.op_begin.size() * 4);
        arr(D[k].o_entry_begin, G.P.entry_begin.size() * 4);
        arr(D[k].o_entries, G.P.entries.size() * 2);
        arr(D[k].o_entry_value, G.P.entry_value.size() * 4);
        arr(D[k].o_lists, G.lists.size() * 4);
        arr(D[k].o_chunk_off, G.chunk_off.size() * 8);
        arr(D[k].o_chunk_len, G.chunk_len.size() * 4);
    }
    L.copy_bytes = img;
    L.ctr_off = img;
    const size_t base = img + 256;  // every phase's regions start here
    size_t ws_end = base;
    for (size_t p = 0; p < nphases; ++p) {
        run_phase &ph = L.phases[p];
        size_t ws = base;
        int64_t tb = 0, cbb = 0, tiles = 0, red = 0, norm = 0;
        std::vector<size_t> ks;
        for (size_t k = 0; k < nd; ++k)
            if (phase_of[k] == p) ks.push_back(k);
        const bool pad = pad_run(ks.size(), [&](size_t q) -> const job & { return pl.jobs[ks[q]]; });
        for (size_t k : ks) {
            const job &G = pl.jobs[k];
            prob_desc &d = D[k];
            const bool pad_k = pad && G.Lj_pad;
            d.m = G.P.m;
            d.n = G.P.n;
            d.l = G.l;
            d.g = G.P.g;
            d.ngroups = G.P.ngroups;
            d.emax = std::max(G.P.max_entries, 1);
            d.rmax = std::max(G.P.max_regs, 1);
            d.c_form = G.c_form;
            d.direct = G.direct ? 1 : 0;
            d.J = G.J;
            d.Lj = pad_k ? G.Lj_pad : G.Lj;
            d.coop_w = pad_k ? G.coop_w : 0;
            if (d.coop_w > 1) ph.coop = true;
            d.coop_lpu = G.coop_lpu;
            d.coop_h = G.coop_h;
            if (d.coop_w > 1) d.rmax = G.coop_slots;
            d.tm = G.tm;
            d.pp = G.pp;
            d.kc = G.kc;
            d.S = G.S;
            d.gps = G.gps;
            d.io = G.index;
            d.tiles_x = G.tiles_x;
            d.tiles_y = G.tiles_y;
            d.norm_per = G.norm_per;
            d.chunks_per_split = G.chunks_per_split;
            d.n_lanes = d.coop_w > 1 ? G.n_lanes_coop : pad_k ? G.n_lanes_pad : G.n_lanes;
            d.nunits = G.P.nunits;
            d.levels = G.P.max_levels;
            d.tb_block0 = tb;
            tb += (d.n_lanes + 255) / 256;
            d.cb_lanes = G.cb_lanes;
            d.cb_block0 = cbb;
            cbb += (G.cb_lanes + 255) / 256;
            d.tile0 = tiles;
            tiles += (int64_t)G.tiles_x * G.tiles_y * G.S;
            d.red_block0 = red;
            d.red_threads = G.S > 1 ? (2 * (int64_t)G.P.m * G.l * std::min(G.S, REDUCE_LANES) + 255) / 256 * 256 : 0;
            red += d.red_threads / 256;
            d.norm_block0 = norm;
            d.norm_threads = G.norm_threads;
            norm += G.norm_threads / 256;
            d.ldj = G.ldj;
            d.ld_pre = G.ld_pre;
            d.w_regs = (int64_t)ws;
            ws += align256(d.coop_w > 1 ? G.regs_bytes_coop : pad_k ? G.regs_bytes_pad : G.regs_bytes);
            d.w_table = (int64_t)ws;
            ws += align256(G.table_bytes);
            d.w_part = (int64_t)ws;
            ws += align256(G.part_bytes);
            d.w_cjac = (int64_t)ws;
            ws += align256(G.cjac_bytes);
            d.w_norm = (int64_t)ws;
            ws += align256(G.norm_bytes);
            d.w_cprod = (int64_t)ws;
            ws += align256(G.cprod_bytes);
            ph.levels = std::max(ph.levels, G.cb_lanes > 0 ? G.P.max_levels : 1);
        }
        ph.tb_blocks = tb;
        ph.cb_blocks = cbb;
        ph.tiles = tiles;
        ph.red_blocks = red;
        ph.norm_blocks = norm;
        ws_end = std::max(ws_end, ws);
        if (tb > 0x7FFFFFFF || cbb > 0x7FFFFFFF || red > 0x7FFFFFFF || norm > 0x7FFFFFFF ||
            tiles > 0x7FFFFFFF - (1 << 20))
            return PCMM_EINVAL;
    }
    L.ws_bytes = ws_end + 256;
    pl.desc = D;
    for (size_t k = 0; k < nd; ++k) pl.stats[pl.jobs[k].index].coop_lanes = D[k].coop_w;
    pl.job_of.assign(pl.count, -1);
    for (size_t k = 0; k < nd; ++k) pl.job_of[pl.jobs[k].index] = (int)k;
    pl.image.assign(img, 0);
    {
        size_t k0 = 0;
        for (size_t p = 0; p < nphases; ++p) {
            const size_t cnt = (size_t)L.phases[p].count;
            memcpy(pl.image.data() + L.phases[p].desc_off, D.data() + k0, cnt * sizeof(prob_desc));
            k0 += cnt;
        }
    }
    for (size_t k = 0; k < nd; ++k) {
        const cussen_plan &P = pl.jobs[k].P;
        auto put = [&](int64_t off, const void *src, size_t bytes) {
            if (bytes) memcpy(pl.image.data() + off, src, bytes);
        };
        put(D[k].o_ops, P.ops.data(), P.ops.size() * sizeof(plan_op));
        put(D[k].o_unit_col, P.unit_col.data(), P.unit_col.size() * 4);
        put(D[k].o_unit_grp, P.unit_grp.data(), P.unit_grp.size() * 4);
        put(D[k].o_unit_off, P.unit_off.data(), P.unit_off.size() * 4);
        put(D[k].o_cblock_begin, P.cblock_begin.data(), P.cblock_begin.size() * 4);
        put(D[k].o_cblocks, P.cblocks.data(), P.cblocks.size() * sizeof(plan_cblock));
        put(D[k].o_cruns, P.cruns.data(), P.cruns.size() * sizeof(plan_crun));
        put(D[k].o_op_begin, P.op_begin.data(), P.op_begin.size() * 4);
        put(D[k].o_entry_begin, P.entry_begin.data(), P.entry_begin.size() * 4);
        put(D[k].o_entries, P.entries.data(), P.entries.size() * 2);
        put(D[k].o_entry_value, P.entry_value.data(), P.entry_value.size() * 4);
        const job &G = pl.jobs[k];
        put(D[k].o_lists, G.lists.data(), G.lists.size() * 4);
        put(D[k].o_chunk_off, G.chunk_off.data(), G.chunk_off.size() * 8);
        put(D[k].o_chunk_len, G.chunk_len.data(), G.chunk_len.size() * 4);
    }
    return PCMM_OK;
}

std::mutex g_occ_lock;
std::map<int, int64_t> g_occ_cache;  // device -> resident workgroups

// Sizes the persistent accumulation grid of each phase of L on `device`
// (current): the workgroups that fit on the device at once, or the phase's
// tiles if fewer.
pcmm_status size_acc_grid(int device, run_layout &L) {
    int64_t cap = 0;
    {
        std::lock_guard<std::mutex> guard(g_occ_lock);
        auto it = g_occ_cache.find(device);
        if (it != g_occ_cache.end()) cap = it->second;
    }
    if (cap == 0 && !L.phases.empty()) {
        int per_cu = 0, cus = 0;
        PCMM_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, accumulate_kernel, 256, 0));
        PCMM_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
        cap = (int64_t)std::max(per_cu, 1) * std::max(cus, 1);
        std::lock_guard<std::mutex> guard(g_occ_lock);
        g_occ_cache[device] = cap;
    }
    for (run_phase &ph : L.phases) ph.acc_grid = (int)std::min<int64_t>(ph.tiles, cap);
    return PCMM_OK;
}

// Binds pl to the current device.
pcmm_status bind_device(pcmm_plan_s &pl) {
    PCMM_HIP_TRY(hipGetDevice(&pl.device));
    return size_acc_grid(pl.device, pl.full);
}

// Compiles problems into pl (host threads over problems; no device calls).
// Returns the first error in problem order.
pcmm_status build_plan(const pcmm_problem *probs, int count, pcmm_plan_s &pl) {
    if (!probs || count < 1 || count > MAX_PROBLEMS) return PCMM_EINVAL;
    for (int i = 0; i < count; ++i) {
        const pcmm_problem &q = probs[i];
        // (the accumulation steps between table entries in 32-bit byte strides)
        if (q.m < 0 || q.n < 0 || q.l < 0 || entry_stride(2 * (int64_t)q.l) * 4 > (int64_t)UINT32_MAX ||
            (q.c_form != PCMM_AFFINE && q.c_form != PCMM_JACOBIAN) ||
            !valid_cfg(&q.cfg))
            return PCMM_EINVAL;
    }
    pl.count = count;
    pl.m.resize(count);
    pl.n.resize(count);
    pl.l.resize(count);
    pl.c_form.resize(count);
    pl.stats.assign(count, pcmm_cussen_stats{});
    std::vector<job> built(count);
    std::vector<int> rcs(count, 0);
    // problems on up to host_threads() threads; a problem's column groups
    // share the threads left over (all of them for a single problem)
    const int nthreads = std::min(count, host_threads());
    const int inner = std::max(1, host_threads() / std::max(nthreads, 1));
    auto work = [&](int i) {
        const pcmm_problem &q = probs[i];
        job &G = built[i];
        int split = 1;
        rcs[i] = build_plan_cfg(q.A, q.m, q.n, q.l, q.bits, q.is_signed != 0, &q.cfg, &G.P, &split, inner);
        if (rcs[i]) return;
        G.index = i;
        G.l = q.l;
        G.c_form = q.c_form;
        make_geometry(G, &q.cfg, split);
        if ((int64_t)q.m * q.l > 0 && q.n > 0) pack_codes(G, inner);
    };
    if (nthreads <= 1) {
        for (int i = 0; i < count; ++i) work(i);
    } else {
        std::atomic<int> next{0};
        std::vector<std::thread> pool;
        for (int t = 0; t < nthreads; ++t)
            pool.emplace_back([&]() {
                for (int i = next++; i < count; i = next++) work(i);
            });
        for (auto &th : pool) th.join();
    }
    for (int i = 0; i < count; ++i) {
        if (rcs[i] == -2) return PCMM_ERANGE;
        if (rcs[i]) return PCMM_EINVAL;
    }
    for (int i = 0; i < count; ++i) {
        const pcmm_problem &q = probs[i];
        pl.m[i] = q.m;
        pl.n[i] = q.n;
        pl.l[i] = q.l;
        pl.c_form[i] = q.c_form;
        fill_stats(built[i], &pl.stats[i]);
        if ((int64_t)q.m * q.l == 0 || q.n == 0) pl.stats[i].workspace_bytes = 0;
        if ((int64_t)q.m * q.l == 0) continue;
        if (q.n == 0) {
            pl.full.fills.push_back(i);
            continue;
        }
        pl.jobs.push_back(std::move(built[i]));
    }
    return finish_plan(pl);
}

pcmm_status check_mats(int m, int n, int l, int c_form, const pcmm_mat *B, const pcmm_mat *C) {
    if (!B || !C) return PCMM_EINVAL;
    if (B->rows != n || B->cols != l || B->npts != 2 || B->form != PCMM_AFFINE) return PCMM_EINVAL;
    if (B->ld < (int64_t)n * l || ((int64_t)n * l > 0 && !B->d)) return PCMM_EINVAL;
    if (C->rows != m || C->cols != l || C->npts != 2 || C->form != c_form) return PCMM_EINVAL;
    if (C->ld < (int64_t)m * l || ((int64_t)m * l > 0 && !C->d)) return PCMM_EINVAL;
    if (B->d == C->d && (int64_t)n * l > 0 && (int64_t)m * l > 0) return PCMM_EINVAL;
    return PCMM_OK;
}

// Queues a run: copies L.copy_bytes from the pinned host block copy_src
// (unchanged until the copy has executed) to the start of the workspace, then
// the kernels of each phase.  plan_base: device base of the plan arrays, or
// null for the workspace itself.  B, C: the run's n_io matrices.  ev:
// PCMM_STAGE_EVENTS events or null (with several phases the stage events
// after the upload bracket the last phase; the earlier phases count as table
// stage).
pcmm_status enqueue_run(const run_layout &L, const void *copy_src, const char *plan_base, const pcmm_mat *B,
                        pcmm_mat *C, int n_io, void *workspace, hipEvent_t *ev, hipStream_t s,
                        hipEvent_t copied) {
    auto rec = [&](int i) -> pcmm_status {
        if (ev) PCMM_HIP_TRY(hipEventRecord(ev[i], s));
        return PCMM_OK;
    };
    pcmm_status st;
#define PCMM_REC(i)                              \
    do {                                         \
        if ((st = rec(i)) != PCMM_OK) return st; \
    } while (0)
    const bool gpu_work = !L.phases.empty();
    PCMM_REC(0);
    run_args ra{};
    if (gpu_work) {
        ra.ws = (char *)workspace;
        ra.plan = plan_base ? plan_base : (const char *)workspace;
        ra.ctr_off = (int64_t)L.ctr_off;
        for (int i = 0; i < n_io; ++i) ra.io[i] = io_ptrs{B[i].d, C[i].d, B[i].ld, C[i].ld};
        PCMM_HIP_TRY(hipMemcpyAsync(workspace, copy_src, L.copy_bytes, hipMemcpyHostToDevice, s));
    }
    // the host buffer may be refilled once its copy has executed, while the
    // kernels below still run
    if (copied) PCMM_HIP_TRY(hipEventRecord(copied, s));
    PCMM_REC(1);
    const size_t nph = L.phases.size();
    for (size_t p = 0; p < nph; ++p) {
        const run_phase &ph = L.phases[p];
        const bool last = p + 1 == nph;
        ra.desc = (const char *)workspace + ph.desc_off;
        ra.count = ph.count;
        ra.total_tiles = ph.tiles;
        // the table build also resets the accumulation's tile counter
        hipLaunchKernelGGL(table_build_kernel, dim3((unsigned)ph.tb_blocks), dim3(256), 0, s, ra);
        PCMM_LAUNCH_CHECK();
        if (ph.coop) {
            hipLaunchKernelGGL(coop_table_kernel, dim3((unsigned)ph.tb_blocks), dim3(256), 0, s, ra);
            PCMM_LAUNCH_CHECK();
        }
        // combinations level by level: a forward kernel (few registers, many
        // wavefronts in flight) and a backward kernel per level
        for (int lev = 2; ph.cb_blocks > 0 && lev <= ph.levels; ++lev) {
            hipLaunchKernelGGL(combo_forward_kernel, dim3((unsigned)ph.cb_blocks), dim3(256), 0, s, ra, lev);
            PCMM_LAUNCH_CHECK();
            hipLaunchKernelGGL(combo_backward_kernel, dim3((unsigned)ph.cb_blocks), dim3(256), 0, s, ra, lev);
            PCMM_LAUNCH_CHECK();
        }
        if (last) PCMM_REC(2);
        hipLaunchKernelGGL(accumulate_kernel, dim3((unsigned)ph.acc_grid), dim3(256), 0, s, ra);
        PCMM_LAUNCH_CHECK();
        if (last) PCMM_REC(3);
        if (ph.red_blocks > 0) {
            hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)ph.red_blocks), dim3(256), 0, s, ra);
            PCMM_LAUNCH_CHECK();
        }
        if (last) PCMM_REC(4);
        if (ph.norm_blocks > 0) {
            hipLaunchKernelGGL(normalize_batch_kernel, dim3((unsigned)ph.norm_blocks), dim3(256), 0, s, ra);
            PCMM_LAUNCH_CHECK();
        }
    }
    if (!gpu_work) {
        PCMM_REC(2);
        PCMM_REC(3);
        PCMM_REC(4);
    }
    for (int i : L.fills) {
        const int64_t n_out = (int64_t)C[i].rows * C[i].cols;
        hipLaunchKernelGGL(fill_infinity_kernel, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, s, C[i].d,
                           C[i].ld, n_out, C[i].form);
        PCMM_LAUNCH_CHECK();
    }
    PCMM_REC(5);
#undef PCMM_REC
    return PCMM_OK;
}

// Matrices of a run of problems which[0..k) of pl (all problems in order
// when which is null) against the workspace it needs.
pcmm_status check_run(const pcmm_plan_s &pl, const int32_t *which, int k, const pcmm_mat *B, pcmm_mat *C,
                      void *workspace, size_t ws_bytes, size_t need, bool gpu_work) {
    if (!B || !C) return PCMM_EINVAL;
    for (int r = 0; r < k; ++r) {
        const int i = which ? which[r] : r;
        pcmm_status st = check_mats(pl.m[i], pl.n[i], pl.l[i], pl.c_form[i], &B[r], &C[r]);
        if (st != PCMM_OK) return st;
    }
    if (gpu_work && (!workspace || ws_bytes < need)) return PCMM_ENOMEM;
    return PCMM_OK;
}

// events bracketing the stages of one profiled call
struct stage_events {
    hipEvent_t e[PCMM_STAGE_EVENTS] = {};
    hipError_t create() {
        for (auto &x : e) {
            hipError_t r = hipEventCreate(&x);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    }
    ~stage_events() {
        for (auto &x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

// pinned staging for the plan image of pcmm_cussen calls: a ring of
// STAGE_RING buffers per device, each guarded by an event recorded after its
// copy, so the host can plan up to STAGE_RING calls ahead of the device (a
// host stall shorter than that many runs leaves the device busy)
constexpr int STAGE_RING = 4;
struct staging {
    void *host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
};
std::mutex g_stage_lock;
staging g_stage[64][STAGE_RING];
int g_stage_next[64];

pcmm_problem single_problem(const void *A, int m, int n, int l, int bits, int is_signed, int c_form,
                            const pcmm_cussen_cfg *cfg) {
    pcmm_problem q{};
    q.A = A;
    q.m = m;
    q.n = n;
    q.l = l;
    q.bits = bits;
    q.is_signed = is_signed;
    q.c_form = c_form;
    if (cfg) q.cfg = *cfg;
    q.cfg.profile = 0;
    q.cfg.stage_events = nullptr;
    return q;
}

}  // namespace

extern "C" pcmm_status pcmm_cussen_plan_stats(const void *A, int32_t m, int32_t n, int32_t bits,
                                              int32_t is_signed, const pcmm_cussen_cfg *cfg,
                                              pcmm_cussen_stats *stats) {
    if (!stats || !valid_cfg(cfg) || m < 0 || n < 0) return PCMM_EINVAL;
    job G;
    int split = 1;
    // without output columns given, the tuner assumes a square problem (l = m)
    int rc = build_plan_cfg(A, m, n, std::max(m, 1), bits, is_signed != 0, cfg, &G.P, &split, host_threads());
    if (rc == -2) return PCMM_ERANGE;
    if (rc) return PCMM_EINVAL;
    G.l = 1;
    make_geometry(G, cfg, split);
    fill_stats(G, stats);
    stats->k_split = 0;
    stats->lanes_per_chain = 0;
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_cussen_workspace(const void *A, int32_t m, int32_t n, int32_t l, int32_t bits,
                                             int32_t is_signed, int32_t c_form, const pcmm_cussen_cfg *cfg,
                                             size_t *bytes) {
    if (!bytes || !valid_cfg(cfg)) return PCMM_EINVAL;
    pcmm_plan_s pl;
    pcmm_problem q = single_problem(A, m, n, l, bits, is_signed, c_form, cfg);
    pcmm_status st = build_plan(&q, 1, pl);
    if (st != PCMM_OK) return st;
    *bytes = pl.full.ws_bytes;
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_cussen(const void *A, int32_t m, int32_t n, int32_t bits, int32_t is_signed,
                                   const pcmm_mat *B, pcmm_mat *C, const pcmm_cussen_cfg *cfg, void *workspace,
                                   size_t ws_bytes, pcmm_cussen_stats *stats, void *stream) {
    if (!B || !C || !valid_cfg(cfg)) return PCMM_EINVAL;
    if (C->form != PCMM_AFFINE && C->form != PCMM_JACOBIAN) return PCMM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t ev[PCMM_STAGE_EVENTS] = {};
    const bool caller_events = cfg && cfg->stage_events;
    if (caller_events) {
        for (int i = 0; i < PCMM_STAGE_EVENTS; ++i) {
            ev[i] = (hipEvent_t)cfg->stage_events[i];
            if (!ev[i]) return PCMM_EINVAL;
        }
    }
    pcmm_plan_s pl;
    pcmm_problem q = single_problem(A, m, n, B->cols, bits, is_signed, C->form, cfg);
    pcmm_status st = build_plan(&q, 1, pl);
    if (st != PCMM_OK) return st;
    if (stats) *stats = pl.stats[0];
    st = check_run(pl, nullptr, 1, B, C, workspace, ws_bytes, pl.full.ws_bytes, !pl.full.phases.empty());
    if (st != PCMM_OK) return st;
    st = bind_device(pl);
    if (st != PCMM_OK) return st;
    const bool wait_prof = cfg && cfg->profile;
    stage_events own;
    if (wait_prof && !caller_events) {
        PCMM_HIP_TRY(own.create());
        for (int i = 0; i < PCMM_STAGE_EVENTS; ++i) ev[i] = own.e[i];
    }
    const bool prof = wait_prof || caller_events;
    {
        // stage the image in the device's pinned buffer, once its previous copy
        // has executed (the previous run's kernels may still be running)
        std::lock_guard<std::mutex> guard(g_stage_lock);
        if (pl.device < 0 || pl.device >= 64) return PCMM_EDEVICE;
        staging &sg = g_stage[pl.device][g_stage_next[pl.device]];
        g_stage_next[pl.device] = (g_stage_next[pl.device] + 1) % STAGE_RING;
        const size_t bytes = std::max<size_t>(pl.image.size(), 256);
        (void)ws_bytes;
        if (sg.done) PCMM_HIP_TRY(hipEventSynchronize(sg.done));
        if (sg.bytes < bytes) {
            if (sg.host) (void)hipHostFree(sg.host);
            sg.host = nullptr;
            sg.bytes = 0;
            PCMM_HIP_TRY(hipHostMalloc(&sg.host, bytes, hipHostMallocDefault));
            sg.bytes = bytes;
        }
        if (!sg.done) PCMM_HIP_TRY(hipEventCreateWithFlags(&sg.done, hipEventDisableTiming));
        if (!pl.image.empty()) memcpy(sg.host, pl.image.data(), pl.image.size());
        st = enqueue_run(pl.full, sg.host, nullptr, B, C, 1, workspace, prof ? ev : nullptr, s, sg.done);
        if (st != PCMM_OK) return st;
    }
    if (wait_prof) {
        PCMM_HIP_TRY(hipEventSynchronize(ev[5]));
        if (stats) {
            float *dst[5] = {&stats->ms_upload, &stats->ms_table, &stats->ms_accumulate, &stats->ms_reduce,
                             &stats->ms_normalize};
            for (int i = 0; i < 5; ++i) PCMM_HIP_TRY(hipEventElapsedTime(dst[i], ev[i], ev[i + 1]));
            PCMM_HIP_TRY(hipEventElapsedTime(&stats->ms_total, ev[0], ev[5]));
        }
    }
    return PCMM_OK;
}

// --------------------------------------------------------------------------
// pcmm_cussen_static: pcmm_cussen with the workspace in a fixed device array
// --------------------------------------------------------------------------
// The library's own scratch for callers that cannot allocate device memory.
// Every GPU the library runs on holds one copy for the life of the process;
// the name is a host-side stand-in, so host code uses only the per-device
// address that hipGetSymbolAddress returns.
__device__ __align__(256) char scratch[PCMM_STATIC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_lock;
void *g_scratch_ptr[64] = {};

// Address of the current device's scratch, looked up once per device with
// that device current.
pcmm_status scratch_of(int device, void **ptr) {
    if (device < 0 || device >= 64) return PCMM_EDEVICE;
    std::lock_guard<std::mutex> guard(g_scratch_lock);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        PCMM_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return PCMM_EDEVICE;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return PCMM_OK;
}

}  // namespace

extern "C" pcmm_status pcmm_cussen_static(const void *A, int32_t m, int32_t n, int32_t bits, int32_t is_signed,
                                          const pcmm_mat *B, pcmm_mat *C, const pcmm_cussen_cfg *cfg,
                                          pcmm_cussen_stats *stats, void *stream) {
    if (!B || !C || !valid_cfg(cfg)) return PCMM_EINVAL;
    if (cfg && cfg->profile) return PCMM_EINVAL;  // profiling would create events
    if (C->form != PCMM_AFFINE && C->form != PCMM_JACOBIAN) return PCMM_EINVAL;
    hipEvent_t ev[PCMM_STAGE_EVENTS] = {};
    const bool caller_events = cfg && cfg->stage_events;
    if (caller_events) {
        for (int i = 0; i < PCMM_STAGE_EVENTS; ++i) {
            ev[i] = (hipEvent_t)cfg->stage_events[i];
            if (!ev[i]) return PCMM_EINVAL;
        }
    }
    pcmm_plan_s pl;
    pcmm_problem q = single_problem(A, m, n, B->cols, bits, is_signed, C->form, cfg);
    pcmm_status st = build_plan(&q, 1, pl);
    if (st != PCMM_OK) return st;
    if (stats) *stats = pl.stats[0];
    const bool gpu_work = !pl.full.phases.empty();
    // the size check comes before any device call
    if (gpu_work && pl.full.ws_bytes > (size_t)PCMM_STATIC_SCRATCH_BYTES) return PCMM_ETOOLARGE;
    st = check_mats(m, n, B->cols, C->form, B, C);
    if (st != PCMM_OK) return st;
    st = bind_device(pl);
    if (st != PCMM_OK) return st;
    void *ws = nullptr;
    st = scratch_of(pl.device, &ws);
    if (st != PCMM_OK) return st;
    // The image is copied from pageable host memory: the copy is ordered
    // after the stream's earlier work (which may still read the scratch) and
    // has consumed the host bytes when the call returns.
    return enqueue_run(pl.full, pl.image.data(), nullptr, B, C, 1, ws, caller_events ? ev : nullptr,
                       (hipStream_t)stream, nullptr);
}

extern "C" pcmm_status pcmm_plan_create(const pcmm_problem *problems, int32_t count, pcmm_plan *out) {
    if (!out) return PCMM_EINVAL;
    *out = nullptr;
    pcmm_plan_s *pl = new (std::nothrow) pcmm_plan_s;
    if (!pl) return PCMM_ENOMEM;
    pcmm_status st;
    try {
        st = build_plan(problems, count, *pl);
    } catch (const std::bad_alloc &) {
        st = PCMM_ENOMEM;
    }
    if (st == PCMM_OK) st = bind_device(*pl);
    if (st == PCMM_OK && !pl->image.empty()) {
        if (hipHostMalloc(&pl->pinned, pl->image.size(), hipHostMallocDefault) != hipSuccess) {
            pl->pinned = nullptr;
            st = PCMM_EDEVICE;
        } else {
            memcpy(pl->pinned, pl->image.data(), pl->image.size());
        }
    }
    if (st != PCMM_OK) {
        delete pl;
        return st;
    }
    *out = pl;
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_plan_destroy(pcmm_plan plan) {
    delete plan;
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_plan_workspace(pcmm_plan plan, size_t *bytes) {
    if (!plan || !bytes) return PCMM_EINVAL;
    *bytes = plan->full.ws_bytes;
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_plan_stats(pcmm_plan plan, int32_t index, pcmm_cussen_stats *stats) {
    if (!plan || !stats || index < 0 || index >= plan->count) return PCMM_EINVAL;
    *stats = plan->stats[index];
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_plan_run(pcmm_plan plan, const pcmm_mat *B, pcmm_mat *C, void *workspace,
                                     size_t ws_bytes, void **stage_events, void *stream) {
    if (!plan) return PCMM_EINVAL;
    int dev = -1;
    PCMM_HIP_TRY(hipGetDevice(&dev));
    if (dev != plan->device) return PCMM_EDEVICE;
    pcmm_status st = check_run(*plan, nullptr, plan->count, B, C, workspace, ws_bytes, plan->full.ws_bytes,
                               !plan->full.phases.empty());
    if (st != PCMM_OK) return st;
    hipEvent_t ev[PCMM_STAGE_EVENTS] = {};
    if (stage_events) {
        for (int i = 0; i < PCMM_STAGE_EVENTS; ++i) {
            ev[i] = (hipEvent_t)stage_events[i];
            if (!ev[i]) return PCMM_EINVAL;
        }
    }
    return enqueue_run(plan->full, plan->pinned, nullptr, B, C, plan->count, workspace, stage_events ? ev : nullptr,
                       (hipStream_t)stream, nullptr);  // the pinned image is immutable
}

namespace {

// Layout and descriptors of a run of problems which[0..k) of pl.
pcmm_status selected_layout(const pcmm_plan_s &pl, const int32_t *which, int k, run_layout &L,
                            std::vector<prob_desc> &D) {
    if (!which || k < 1 || k > MAX_PROBLEMS) return PCMM_EINVAL;
    std::vector<int> order;
    L = run_layout{};
    for (int r = 0; r < k; ++r) {
        const int i = which[r];
        if (i < 0 || i >= pl.count) return PCMM_EINVAL;
        if (pl.job_of[i] >= 0) order.push_back(r);
        else if ((int64_t)pl.m[i] * pl.l[i] > 0 && pl.n[i] == 0) L.fills.push_back(r);
    }
    // most expensive accumulation tiles first
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return pl.jobs[pl.job_of[which[x]]].tile_cost > pl.jobs[pl.job_of[which[y]]].tile_cost;
    });
    const size_t nd = order.size();
    if (nd > 0) L.phases.assign(1, run_phase{});
    run_phase dummy;
    run_phase &ph = nd > 0 ? L.phases[0] : dummy;
    ph.count = (int32_t)nd;
    ph.desc_off = 0;
    L.copy_bytes = align256(nd * sizeof(prob_desc));
    L.ctr_off = L.copy_bytes;
    size_t ws = L.ctr_off + 256;
    D.resize(nd);
    int64_t tb = 0, cbb = 0, tiles = 0, red = 0, norm = 0;
    const bool pad = pad_run(nd, [&](size_t q) -> const job & { return pl.jobs[pl.job_of[which[order[q]]]]; });
    for (size_t q = 0; q < nd; ++q) {
        const int r = order[q];
        const int jk = pl.job_of[which[r]];
        const job &G = pl.jobs[jk];
        prob_desc d = pl.desc[jk];
        const bool pad_k = pad && G.Lj_pad;
        d.Lj = pad_k ? G.Lj_pad : G.Lj;
        d.coop_w = pad_k ? G.coop_w : 0;
        if (d.coop_w > 1) ph.coop = true;
        d.coop_lpu = G.coop_lpu;
        d.coop_h = G.coop_h;
        d.rmax = d.coop_w > 1 ? G.coop_slots : std::max(G.P.max_regs, 1);
        d.n_lanes = d.coop_w > 1 ? G.n_lanes_coop : pad_k ? G.n_lanes_pad : G.n_lanes;
        d.io = r;
        d.tb_block0 = tb;
        tb += (d.n_lanes + 255) / 256;
        d.cb_block0 = cbb;
        cbb += (d.cb_lanes + 255) / 256;
        d.tile0 = tiles;
        tiles += (int64_t)G.tiles_x * G.tiles_y * G.S;
        d.red_block0 = red;
        red += d.red_threads / 256;
        d.norm_block0 = norm;
        norm += d.norm_threads / 256;
        d.w_regs = (int64_t)ws;
        ws += align256(d.coop_w > 1 ? G.regs_bytes_coop : pad_k ? G.regs_bytes_pad : G.regs_bytes);
        d.w_table = (int64_t)ws;
        ws += align256(G.table_bytes);
        d.w_part = (int64_t)ws;
        ws += align256(G.part_bytes);
        d.w_cjac = (int64_t)ws;
        ws += align256(G.cjac_bytes);
        d.w_norm = (int64_t)ws;
        ws += align256(G.norm_bytes);
        d.w_cprod = (int64_t)ws;
        ws += align256(G.cprod_bytes);
        ph.levels = std::max(ph.levels, G.cb_lanes > 0 ? G.P.max_levels : 1);
        D[q] = d;
    }
    L.ws_bytes = ws + 256;
    ph.tb_blocks = tb;
    ph.cb_blocks = cbb;
    ph.tiles = tiles;
    ph.red_blocks = red;
    ph.norm_blocks = norm;
    return PCMM_OK;
}

constexpr int RING_SLOTS = 8;

}  // namespace

extern "C" pcmm_status pcmm_plan_resident_bytes(pcmm_plan plan, size_t *bytes) {
    if (!plan || !bytes) return PCMM_EINVAL;
    *bytes = std::max<size_t>(plan->image.size(), 256);
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_plan_make_resident(pcmm_plan plan, void *device_mem, size_t bytes, void *stream) {
    if (!plan || !device_mem || bytes < std::max<size_t>(plan->image.size(), 256)) return PCMM_EINVAL;
    int dev = -1;
    PCMM_HIP_TRY(hipGetDevice(&dev));
    if (dev != plan->device) return PCMM_EDEVICE;
    if (!plan->image.empty())
        PCMM_HIP_TRY(hipMemcpyAsync(device_mem, plan->pinned, plan->image.size(), hipMemcpyHostToDevice,
                                    (hipStream_t)stream));
    plan->resident = (const char *)device_mem;
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_plan_selected_workspace(pcmm_plan plan, const int32_t *which, int32_t k,
                                                    size_t *bytes) {
    if (!plan || !bytes) return PCMM_EINVAL;
    run_layout L;
    std::vector<prob_desc> D;
    pcmm_status st = selected_layout(*plan, which, k, L, D);
    if (st != PCMM_OK) return st;
    *bytes = L.ws_bytes;
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_plan_run_selected(pcmm_plan plan, const int32_t *which, int32_t k, const pcmm_mat *B,
                                              pcmm_mat *C, void *workspace, size_t ws_bytes, void **stage_events,
                                              void *stream) {
    if (!plan || !plan->resident) return PCMM_EINVAL;
    int dev = -1;
    PCMM_HIP_TRY(hipGetDevice(&dev));
    if (dev != plan->device) return PCMM_EDEVICE;
    run_layout L;
    std::vector<prob_desc> D;
    pcmm_status st = selected_layout(*plan, which, k, L, D);
    if (st != PCMM_OK) return st;
    st = check_run(*plan, which, k, B, C, workspace, ws_bytes, L.ws_bytes, !L.phases.empty());
    if (st != PCMM_OK) return st;
    hipEvent_t ev[PCMM_STAGE_EVENTS] = {};
    if (stage_events) {
        for (int i = 0; i < PCMM_STAGE_EVENTS; ++i) {
            ev[i] = (hipEvent_t)stage_events[i];
            if (!ev[i]) return PCMM_EINVAL;
        }
    }
    st = size_acc_grid(plan->device, L);
    if (st != PCMM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> guard(plan->stage_lock);
    if (plan->ring.empty()) plan->ring.resize(RING_SLOTS);
    stage_slot &slot = plan->ring[plan->ring_next];
    plan->ring_next = (plan->ring_next + 1) % RING_SLOTS;
    if (!slot.host) {
        PCMM_HIP_TRY(hipHostMalloc(&slot.host, align256(MAX_PROBLEMS * sizeof(prob_desc)), hipHostMallocDefault));
        PCMM_HIP_TRY(hipEventCreateWithFlags(&slot.done, hipEventDisableTiming));
    } else {
        PCMM_HIP_TRY(hipEventSynchronize(slot.done));
    }
    if (!D.empty()) memcpy(slot.host, D.data(), D.size() * sizeof(prob_desc));
    return enqueue_run(L, slot.host, plan->resident, B, C, k, workspace, stage_events ? ev : nullptr, s, slot.done);
}
