// k_cussen.hip -- Cussen PC-MM (Alg. 3 with Alg. 2) on gfx950.
//
// Three kernels:
//   table_build   one lane per (column group, J output columns j, point): runs
//                 the group's straight-line program (level-N ladders, prefix
//                 sums, digit combinations) on B[k0.., j], keeps every
//                 register in a lane-private scratch (structure of arrays, so
//                 the lanes' accesses coalesce), then converts its tables to
//                 affine with one inversion for all of its J tables.
//   accumulate    C_ij += sign * T_kj[code_ik]: each workgroup stages the tables
//                 of a chunk of column groups for its (j, point) pairs in LDS;
//                 every lane owns one accumulator (row i, pair) in VGPRs and
//                 walks the chunk with mixed additions.  The inner dimension
//                 may be split over independent partial sums.
//   reduce        adds the split-k partial sums of one output with a tree of
//                 point additions across the lanes of a wavefront (shuffles).
#include <mutex>
#include <vector>

#include "common.hpp"
#include "normalize.hpp"
#include "plan.hpp"

using namespace pcmm;

namespace {

constexpr int ENTRY_WORDS = 20;  // affine entry: x (9 limbs), y (9 limbs), 2 pad words; Montgomery form

struct tb_args {
    const plan_op *ops;
    const int32_t *op_begin;
    const int32_t *entry_begin;
    const int16_t *entries;
    const uint32_t *B;  // n x l ciphertexts, affine canonical
    int64_t ldb;
    int n, l, g, J, Lj, rmax, emax;
    int64_t n_lanes;
    uint32_t *regs;     // [(r * rmax + reg) * 27 + word][lane]
    uint32_t *table;    // [((grp * l + j) * 2 + pt) * emax + e][ENTRY_WORDS]
};

constexpr int JAC_WORDS = 3 * NL;

__device__ __forceinline__ jpt reg_load(const tb_args &a, int r, int reg, int64_t lane) {
    return load_jac_m(a.regs + (int64_t)(r * a.rmax + reg) * JAC_WORDS * a.n_lanes, a.n_lanes, 0, lane);
}

__device__ __forceinline__ void reg_store(const tb_args &a, int r, int reg, int64_t lane, const jpt &P) {
    store_jac_m(a.regs + (int64_t)(r * a.rmax + reg) * JAC_WORDS * a.n_lanes, a.n_lanes, 0, lane, P);
}

__device__ __forceinline__ apt base_point(const apt Bt[4], int t) {
    apt r = Bt[0];
    if (t == 1) r = Bt[1];
    if (t == 2) r = Bt[2];
    if (t == 3) r = Bt[3];
    return r;
}

__global__ void __launch_bounds__(256) table_build_kernel(tb_args a) {
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= a.n_lanes) return;
    const int lanes_per_group = 2 * a.Lj;
    const int grp = (int)(lane / lanes_per_group);
    const int rem = (int)(lane % lanes_per_group);
    const int jslot = rem >> 1;
    const int pt = rem & 1;
    const int k0 = grp * a.g;
    const int gg = min(a.g, a.n - k0);
    const int ob = a.op_begin[grp], oe = a.op_begin[grp + 1];
    const int eb = a.entry_begin[grp], ee = a.entry_begin[grp + 1];
    const int E = ee - eb;

    fe prod = fe_one_mont();
    int last_r = -1;
    for (int r = 0; r < a.J; ++r) {
        const int j = jslot + r * a.Lj;
        if (j >= a.l) break;
        last_r = r;
        apt Bt[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t < gg) Bt[t] = load_affine(a.B, a.ldb, pt, (int64_t)(k0 + t) * a.l + j);
            else Bt[t] = Bt[0];
        }
        for (int o = ob; o < oe; ++o) {
            const plan_op op = a.ops[o];
            jpt R;
            if (op.kind == OP_MUL) {
                int s = op.s;
                int bits = 32 - __builtin_clz((unsigned)s);
                R = ladder_small((uint32_t)s, bits, base_point(Bt, -1 - op.a));
            } else {
                if (op.a >= 0 && op.b >= 0) {
                    jpt Q = reg_load(a, r, op.b, lane);
                    if (op.neg_b) Q = jpt_neg(Q);
                    R = jpt_add(reg_load(a, r, op.a, lane), Q);
                } else if (op.b < 0) {
                    apt Q = base_point(Bt, -1 - op.b);
                    if (op.neg_b) Q = apt_neg(Q);
                    jpt P = op.a >= 0 ? reg_load(a, r, op.a, lane) : jpt_from_affine(base_point(Bt, -1 - op.a));
                    R = jpt_add_affine(P, Q);
                } else {
                    // a is a base point, b a register: a + (+-b) = (+-b) + a
                    jpt Q = reg_load(a, r, op.b, lane);
                    if (op.neg_b) Q = jpt_neg(Q);
                    R = jpt_add_affine(Q, base_point(Bt, -1 - op.a));
                }
            }
            reg_store(a, r, op.dst, lane, R);
        }
        // forward pass of the batched inversion over this table's register entries
        const int64_t T = ((int64_t)grp * a.l + j) * 2 + pt;
        for (int e = 0; e < E; ++e) {
            const int16_t opd = a.entries[eb + e];
            if (opd < 0) continue;
            fe z = reg_load(a, r, opd, lane).Z;
            uint32_t *slot = a.table + (T * a.emax + e) * ENTRY_WORDS;
#pragma unroll
            for (int w = 0; w < NL; ++w) slot[w] = prod.v[w];
            if (!fe_is_zero(z)) prod = fe_mul(prod, z);
        }
    }
    if (last_r < 0) return;
    fe inv = fe_inv(prod);
    for (int r = last_r; r >= 0; --r) {
        const int j = jslot + r * a.Lj;
        const int64_t T = ((int64_t)grp * a.l + j) * 2 + pt;
        for (int e = E - 1; e >= 0; --e) {
            const int16_t opd = a.entries[eb + e];
            uint32_t *slot = a.table + (T * a.emax + e) * ENTRY_WORDS;
            apt A;
            if (opd < 0) {
                A = load_affine(a.B, a.ldb, pt, (int64_t)(k0 + (-1 - opd)) * a.l + j);
            } else {
                jpt P = reg_load(a, r, opd, lane);
                fe pre;
#pragma unroll
                for (int w = 0; w < NL; ++w) pre.v[w] = slot[w];
                if (fe_is_zero(P.Z)) {
                    A.x = fe_zero();
                    A.y = fe_zero();
                } else {
                    fe zinv = fe_mul(inv, pre);
                    inv = fe_mul(inv, P.Z);
                    A = jpt_to_affine_with(P, zinv);
                }
            }
#pragma unroll
            for (int w = 0; w < NL; ++w) {
                slot[w] = A.x.v[w];
                slot[NL + w] = A.y.v[w];
            }
        }
    }
}

// --------------------------------------------------------------------------
// Accumulation
// --------------------------------------------------------------------------
struct acc_args {
    const uint32_t *table;   // affine Montgomery entries
    const int16_t *codes;    // [grp * m + i]
    int m, l, ngroups, emax;
    int tm, pp;              // rows and (j, point) pairs per workgroup (tm * pp = 256)
    int kc;                  // groups staged per LDS chunk
    int groups_per_split;
    uint32_t *out;           // Jacobian, Montgomery: partial sums or C
    int64_t ld_out;
    int out_canonical;       // store canonical limbs (C given as Jacobian) instead of Montgomery
};

__global__ void __launch_bounds__(256) accumulate_kernel(acc_args a) {
    extern __shared__ uint32_t lds[];
    const int tid = threadIdx.x;
    const int row_l = tid % a.tm;
    const int pair_l = tid / a.tm;
    const int i = blockIdx.x * a.tm + row_l;
    const int p0 = blockIdx.y * a.pp;
    const int p = p0 + pair_l;
    const int npairs = 2 * a.l;
    const bool active = i < a.m && p < npairs;
    const int split = blockIdx.z;
    const int g_begin = split * a.groups_per_split;
    const int g_end = min(a.ngroups, g_begin + a.groups_per_split);
    const int pairs_here = min(a.pp, npairs - p0);
    const int chunk_words_per_group = a.pp * a.emax * ENTRY_WORDS;

    jpt acc = jpt_infinity();
    for (int gc = g_begin; gc < g_end; gc += a.kc) {
        const int kn = min(a.kc, g_end - gc);
        // stage the tables of groups gc .. gc+kn-1 for pairs p0 .. p0+pairs_here-1
        __syncthreads();
        for (int kk = 0; kk < kn; ++kk) {
            const uint4 *src =
                (const uint4 *)(a.table + ((int64_t)(gc + kk) * npairs + p0) * a.emax * ENTRY_WORDS);
            uint4 *dst = (uint4 *)(lds + (int64_t)kk * chunk_words_per_group);
            const int n4 = pairs_here * a.emax * ENTRY_WORDS / 4;
            for (int x = tid; x < n4; x += blockDim.x) dst[x] = src[x];
        }
        __syncthreads();
        if (active) {
            for (int kk = 0; kk < kn; ++kk) {
                const int code = a.codes[(int64_t)(gc + kk) * a.m + i];
                if (code == 0) continue;
                const int e = (code < 0 ? -code : code) - 1;
                const uint32_t *ent = lds + (int64_t)kk * chunk_words_per_group +
                                      ((int64_t)pair_l * a.emax + e) * ENTRY_WORDS;
                apt Q;
#pragma unroll
                for (int w = 0; w < NL; ++w) {
                    Q.x.v[w] = ent[w];
                    Q.y.v[w] = ent[NL + w];
                }
                if (code < 0) Q.y = fe_neg(Q.y);
                acc = jpt_add_affine(acc, Q);
            }
        }
    }
    if (!active) return;
    const int j = p >> 1, pt = p & 1;
    const int64_t e_out = (int64_t)i * a.l + j;
    uint32_t *dst = a.out + (int64_t)split * JAC2_PLANES * a.ld_out;
    if (a.out_canonical) store_jac(dst, a.ld_out, pt, e_out, acc);
    else store_jac_m(dst, a.ld_out, pt, e_out, acc);
}

// sum of S (power of two <= 64) partial sums per output point; lanes s of one
// output are consecutive
__global__ void __launch_bounds__(256) reduce_kernel(const uint32_t *__restrict__ part, int64_t ld_part, int S,
                                                     int64_t n_out, uint32_t *__restrict__ out, int64_t ld_out,
                                                     int out_canonical) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = (int)(t % S);
    const int64_t rest = t / S;  // (e, pt) pairs, pt fastest
    const bool valid = rest < 2 * n_out;
    const int64_t e = valid ? rest >> 1 : 0;
    const int pt = (int)(rest & 1);
    jpt P = valid ? load_jac_m(part + (int64_t)s * JAC2_PLANES * ld_part, ld_part, pt, e) : jpt_infinity();
    for (int off = S >> 1; off >= 1; off >>= 1) {
        jpt Q;
#pragma unroll
        for (int w = 0; w < NL; ++w) {
            Q.X.v[w] = __shfl_down(P.X.v[w], off, 64);
            Q.Y.v[w] = __shfl_down(P.Y.v[w], off, 64);
            Q.Z.v[w] = __shfl_down(P.Z.v[w], off, 64);
        }
        jpt R = jpt_add(P, Q);
        if (s < off) P = R;
    }
    if (valid && s == 0) {
        if (out_canonical) store_jac(out, ld_out, pt, e, P);
        else store_jac_m(out, ld_out, pt, e, P);
    }
}

// --------------------------------------------------------------------------
// Host side
// --------------------------------------------------------------------------
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct geometry {
    int J, Lj;
    int64_t n_lanes;
    int tm, pp, kc, S, groups_per_split;
    size_t lds_bytes;
    // workspace layout (byte offsets)
    size_t off_plan, off_regs, off_table, off_part, off_cjac, off_norm, total;
    size_t plan_bytes;
};

bool valid_cfg(const pcmm_cussen_cfg *cfg) {
    if (!cfg) return true;
    if (cfg->rounds < 0 || cfg->rounds > 8 || cfg->group < 0 || cfg->group > 4 || cfg->k_split < 0 ||
        cfg->k_split > 64 || cfg->k_chunk < 0 || cfg->profile < 0)
        return false;
    if (cfg->k_split > 0 && (cfg->k_split & (cfg->k_split - 1))) return false;
    return true;
}

int cfg_rounds(const pcmm_cussen_cfg *cfg) { return cfg && cfg->rounds > 0 ? cfg->rounds : 4; }
int cfg_group(const pcmm_cussen_cfg *cfg) { return cfg && cfg->group > 0 ? cfg->group : 1; }

size_t plan_device_bytes(const cussen_plan &P) {
    return align256(P.ops.size() * sizeof(plan_op)) + align256(P.op_begin.size() * 4) +
           align256(P.entry_begin.size() * 4) + align256(P.entries.size() * 2) + align256(P.codes.size() * 2);
}

geometry make_geometry(const cussen_plan &P, int l, int c_form, const pcmm_cussen_cfg *cfg) {
    geometry G{};
    const int m = P.m;
    const int emax = std::max(P.max_entries, 1);
    // table build: J chains per lane so that one inversion serves >= ~64 entries,
    // while keeping >= ~16K lanes
    double avg_e = P.ngroups ? (double)P.table_entries / P.ngroups : 1.0;
    int J = 1;
    while (J < 8 && 2.0 * J * std::max(avg_e, 1.0) <= 64.0) J *= 2;
    while (J > 1 && (int64_t)P.ngroups * 2 * ((l + J - 1) / J) < 16384) J /= 2;
    G.J = J;
    G.Lj = (l + J - 1) / J;
    // lanes of one group fill whole wavefronts (uniform control flow) when possible
    if (2 * G.Lj >= 64) G.Lj = (G.Lj + 31) / 32 * 32;
    G.n_lanes = (int64_t)P.ngroups * 2 * G.Lj;
    // accumulation tile
    const int npairs = 2 * l;
    G.tm = m >= 256 ? 256 : (m > 128 ? 256 : (m > 64 ? 128 : 64));
    G.pp = 256 / G.tm;
    const int64_t wg_base = (int64_t)((m + G.tm - 1) / G.tm) * ((npairs + G.pp - 1) / G.pp);
    const size_t group_bytes = (size_t)G.pp * emax * ENTRY_WORDS * 4;
    int kc = cfg && cfg->k_chunk > 0 ? cfg->k_chunk : (int)std::max<size_t>(1, (64 * 1024) / group_bytes);
    kc = std::max(1, std::min(kc, std::max(P.ngroups, 1)));
    while (kc > 1 && (size_t)kc * group_bytes > 150 * 1024) --kc;
    G.kc = kc;
    G.lds_bytes = (size_t)kc * group_bytes;
    int S = cfg && cfg->k_split > 0 ? cfg->k_split : 1;
    if (!(cfg && cfg->k_split > 0)) {
        while (S < 64 && wg_base * S * 2 <= 2048 && (P.ngroups / (S * 2)) >= 4) S *= 2;
    }
    while (S > 1 && (P.ngroups + S - 1) / S < 1) S /= 2;
    G.S = S;
    G.groups_per_split = P.ngroups > 0 ? (P.ngroups + S - 1) / S : 0;
    // workspace layout
    const int64_t ldc = std::max<int64_t>(64, ((int64_t)m * l + 63) / 64 * 64);
    G.plan_bytes = plan_device_bytes(P);
    G.off_plan = 0;
    G.off_regs = align256(G.plan_bytes);
    size_t regs_bytes = (size_t)G.J * std::max(P.max_regs, 1) * JAC_WORDS * 4 * (size_t)G.n_lanes;
    G.off_table = G.off_regs + align256(regs_bytes);
    size_t table_bytes = (size_t)P.ngroups * npairs * emax * ENTRY_WORDS * 4;
    G.off_part = G.off_table + align256(table_bytes);
    size_t part_bytes = S > 1 ? (size_t)S * JAC2_PLANES * ldc * 4 : 0;
    G.off_cjac = G.off_part + align256(part_bytes);
    size_t cjac_bytes = c_form == PCMM_AFFINE ? (size_t)JAC2_PLANES * ldc * 4 : 0;
    G.off_norm = G.off_cjac + align256(cjac_bytes);
    size_t norm_bytes = c_form == PCMM_AFFINE ? normalize_scratch_bytes((int64_t)m * l, 2) : 0;
    G.total = G.off_norm + align256(norm_bytes) + 256;
    return G;
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
            if (x) hipEventDestroy(x);
    }
};

// pinned staging for plan uploads, one per device; an event guards reuse
struct staging {
    void *host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
};
std::mutex g_stage_lock;
staging g_stage[64];

pcmm_status upload_plan(const cussen_plan &P, void *dev, hipStream_t s) {
    int devid = 0;
    PCMM_HIP_TRY(hipGetDevice(&devid));
    if (devid < 0 || devid >= 64) return PCMM_EDEVICE;
    const size_t bytes = plan_device_bytes(P);
    std::lock_guard<std::mutex> guard(g_stage_lock);
    staging &st = g_stage[devid];
    if (st.done) PCMM_HIP_TRY(hipEventSynchronize(st.done));
    if (st.bytes < bytes) {
        if (st.host) hipHostFree(st.host);
        st.host = nullptr;
        st.bytes = 0;
        PCMM_HIP_TRY(hipHostMalloc(&st.host, bytes, hipHostMallocDefault));
        st.bytes = bytes;
    }
    if (!st.done) PCMM_HIP_TRY(hipEventCreateWithFlags(&st.done, hipEventDisableTiming));
    char *h = (char *)st.host;
    size_t off = 0;
    auto put = [&](const void *src, size_t n) {
        if (n) memcpy(h + off, src, n);
        off += align256(n);
    };
    put(P.ops.data(), P.ops.size() * sizeof(plan_op));
    put(P.op_begin.data(), P.op_begin.size() * 4);
    put(P.entry_begin.data(), P.entry_begin.size() * 4);
    put(P.entries.data(), P.entries.size() * 2);
    put(P.codes.data(), P.codes.size() * 2);
    PCMM_HIP_TRY(hipMemcpyAsync(dev, st.host, bytes, hipMemcpyHostToDevice, s));
    PCMM_HIP_TRY(hipEventRecord(st.done, s));
    return PCMM_OK;
}

pcmm_status check_mats(int m, int n, const pcmm_mat *B, const pcmm_mat *C) {
    if (!B || !C || m < 0 || n < 0) return PCMM_EINVAL;
    if (B->rows != n || B->cols < 0 || B->npts != 2 || B->form != PCMM_AFFINE) return PCMM_EINVAL;
    const int l = B->cols;
    if (B->ld < (int64_t)n * l || ((int64_t)n * l > 0 && !B->d)) return PCMM_EINVAL;
    if (C->rows != m || C->cols != l || C->npts != 2 || (C->form != PCMM_AFFINE && C->form != PCMM_JACOBIAN))
        return PCMM_EINVAL;
    if (C->ld < (int64_t)m * l || ((int64_t)m * l > 0 && !C->d)) return PCMM_EINVAL;
    if (B->d == C->d && (int64_t)n * l > 0 && (int64_t)m * l > 0) return PCMM_EINVAL;
    return PCMM_OK;
}

void fill_stats(const cussen_plan &P, pcmm_cussen_stats *st) {
    if (!st) return;
    memset(st, 0, sizeof *st);
    st->level_mults = P.level_mults;
    st->level_adds = P.level_adds;
    st->table_entries = P.table_entries;
    st->table_adds = P.table_adds;
    st->accum_adds = P.accum_adds;
    st->max_entries = P.max_entries;
}

__global__ void fill_infinity_kernel(uint32_t *out, int64_t ld, int64_t n, int form) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    for (int pt = 0; pt < 2; ++pt)
        for (int c = 0; c < form; ++c)
            for (int w = 0; w < 8; ++w) out[((int64_t)(pt * form + c) * 8 + w) * ld + e] = 0u;
}

}  // namespace

extern "C" pcmm_status pcmm_cussen_plan_stats(const int8_t *A, int32_t m, int32_t n, int32_t bits,
                                              int32_t is_signed, const pcmm_cussen_cfg *cfg,
                                              pcmm_cussen_stats *stats) {
    if (!stats || !valid_cfg(cfg)) return PCMM_EINVAL;
    cussen_plan P;
    int rc = build_cussen_plan(A, m, n, bits, is_signed != 0, cfg_rounds(cfg), cfg_group(cfg), &P);
    if (rc == -2) return PCMM_ERANGE;
    if (rc) return PCMM_EINVAL;
    fill_stats(P, stats);
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_cussen_workspace(const int8_t *A, int32_t m, int32_t n, int32_t l, int32_t bits,
                                             int32_t is_signed, int32_t c_form, const pcmm_cussen_cfg *cfg,
                                             size_t *bytes) {
    if (!bytes || l < 0 || !valid_cfg(cfg) || (c_form != PCMM_AFFINE && c_form != PCMM_JACOBIAN))
        return PCMM_EINVAL;
    cussen_plan P;
    int rc = build_cussen_plan(A, m, n, bits, is_signed != 0, cfg_rounds(cfg), cfg_group(cfg), &P);
    if (rc == -2) return PCMM_ERANGE;
    if (rc) return PCMM_EINVAL;
    *bytes = make_geometry(P, l, c_form, cfg).total;
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_cussen(const int8_t *A, int32_t m, int32_t n, int32_t bits, int32_t is_signed,
                                   const pcmm_mat *B, pcmm_mat *C, const pcmm_cussen_cfg *cfg, void *workspace,
                                   size_t ws_bytes, pcmm_cussen_stats *stats, void *stream) {
    pcmm_status st = check_mats(m, n, B, C);
    if (st != PCMM_OK) return st;
    if (!valid_cfg(cfg)) return PCMM_EINVAL;
    const int l = B->cols;
    hipStream_t s = (hipStream_t)stream;
    cussen_plan P;
    int rc = build_cussen_plan(A, m, n, bits, is_signed != 0, cfg_rounds(cfg), cfg_group(cfg), &P);
    if (rc == -2) return PCMM_ERANGE;
    if (rc) return PCMM_EINVAL;
    fill_stats(P, stats);
    hipEvent_t ev[PCMM_STAGE_EVENTS] = {};
    const bool caller_events = cfg && cfg->stage_events;
    if (caller_events) {
        for (int i = 0; i < PCMM_STAGE_EVENTS; ++i) {
            ev[i] = (hipEvent_t)cfg->stage_events[i];
            if (!ev[i]) return PCMM_EINVAL;
        }
    }
    // calls without the stage pipeline still mark every caller event
    auto record_all = [&]() -> pcmm_status {
        if (caller_events)
            for (int i = 0; i < PCMM_STAGE_EVENTS; ++i) PCMM_HIP_TRY(hipEventRecord(ev[i], s));
        return PCMM_OK;
    };
    const int64_t n_out = (int64_t)m * l;
    if (n_out == 0) return record_all();
    if (n == 0) {
        // empty inner dimension: every output is the identity
        int64_t blocks = (n_out + 255) / 256;
        hipLaunchKernelGGL(fill_infinity_kernel, dim3((unsigned)blocks), dim3(256), 0, s, C->d, C->ld, n_out,
                           C->form);
        PCMM_LAUNCH_CHECK();
        return record_all();
    }
    geometry G = make_geometry(P, l, C->form, cfg);
    if (!workspace || ws_bytes < G.total) return PCMM_ENOMEM;
    if (stats) {
        stats->k_split = G.S;
        stats->lanes_per_chain = G.J;
    }
    char *ws = (char *)workspace;
    const bool wait_prof = cfg && cfg->profile;
    const bool prof = wait_prof || caller_events;
    stage_events own;
    if (wait_prof && !caller_events) {
        PCMM_HIP_TRY(own.create());
        for (int i = 0; i < PCMM_STAGE_EVENTS; ++i) ev[i] = own.e[i];
    }
    if (prof) PCMM_HIP_TRY(hipEventRecord(ev[0], s));
    st = upload_plan(P, ws + G.off_plan, s);
    if (st != PCMM_OK) return st;
    if (prof) PCMM_HIP_TRY(hipEventRecord(ev[1], s));
    // device views of the plan
    size_t off = 0;
    auto view = [&](size_t n_bytes) {
        char *p = ws + G.off_plan + off;
        off += align256(n_bytes);
        return p;
    };
    const plan_op *d_ops = (const plan_op *)view(P.ops.size() * sizeof(plan_op));
    const int32_t *d_op_begin = (const int32_t *)view(P.op_begin.size() * 4);
    const int32_t *d_entry_begin = (const int32_t *)view(P.entry_begin.size() * 4);
    const int16_t *d_entries = (const int16_t *)view(P.entries.size() * 2);
    const int16_t *d_codes = (const int16_t *)view(P.codes.size() * 2);
    const int emax = std::max(P.max_entries, 1);

    tb_args ta;
    ta.ops = d_ops;
    ta.op_begin = d_op_begin;
    ta.entry_begin = d_entry_begin;
    ta.entries = d_entries;
    ta.B = B->d;
    ta.ldb = B->ld;
    ta.n = n;
    ta.l = l;
    ta.g = P.g;
    ta.J = G.J;
    ta.Lj = G.Lj;
    ta.rmax = std::max(P.max_regs, 1);
    ta.emax = emax;
    ta.n_lanes = G.n_lanes;
    ta.regs = (uint32_t *)(ws + G.off_regs);
    ta.table = (uint32_t *)(ws + G.off_table);
    {
        int64_t blocks = (G.n_lanes + 255) / 256;
        hipLaunchKernelGGL(table_build_kernel, dim3((unsigned)blocks), dim3(256), 0, s, ta);
        PCMM_LAUNCH_CHECK();
    }
    if (prof) PCMM_HIP_TRY(hipEventRecord(ev[2], s));
    const int64_t ldc = std::max<int64_t>(64, (n_out + 63) / 64 * 64);
    const bool affine_out = C->form == PCMM_AFFINE;
    uint32_t *jac_out = affine_out ? (uint32_t *)(ws + G.off_cjac) : C->d;
    const int64_t ld_jac = affine_out ? ldc : C->ld;
    acc_args aa;
    aa.table = ta.table;
    aa.codes = d_codes;
    aa.m = m;
    aa.l = l;
    aa.ngroups = P.ngroups;
    aa.emax = emax;
    aa.tm = G.tm;
    aa.pp = G.pp;
    aa.kc = G.kc;
    aa.groups_per_split = G.groups_per_split;
    if (G.S > 1) {
        aa.out = (uint32_t *)(ws + G.off_part);
        aa.ld_out = ldc;
        aa.out_canonical = 0;
    } else {
        aa.out = jac_out;
        aa.ld_out = ld_jac;
        aa.out_canonical = affine_out ? 0 : 1;
    }
    {
        dim3 grid((unsigned)((m + G.tm - 1) / G.tm), (unsigned)((2 * l + G.pp - 1) / G.pp), (unsigned)G.S);
        if (G.lds_bytes > 64 * 1024)
            PCMM_HIP_TRY(hipFuncSetAttribute((const void *)accumulate_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)G.lds_bytes));
        hipLaunchKernelGGL(accumulate_kernel, grid, dim3(256), G.lds_bytes, s, aa);
        PCMM_LAUNCH_CHECK();
    }
    if (prof) PCMM_HIP_TRY(hipEventRecord(ev[3], s));
    if (G.S > 1) {
        int64_t threads = 2 * n_out * G.S;
        int64_t blocks = (threads + 255) / 256;
        hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (const uint32_t *)aa.out, ldc,
                           G.S, n_out, jac_out, ld_jac, affine_out ? 0 : 1);
        PCMM_LAUNCH_CHECK();
    }
    if (prof) PCMM_HIP_TRY(hipEventRecord(ev[4], s));
    if (affine_out) {
        st = launch_normalize(jac_out, ld_jac, true, C->d, C->ld, false, n_out, 2, ws + G.off_norm,
                              G.total - G.off_norm, s);
        if (st != PCMM_OK) return st;
    }
    if (prof) PCMM_HIP_TRY(hipEventRecord(ev[5], s));
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
