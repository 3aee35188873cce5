// plan.cpp -- Alg. 2 compression of the columns of A into table-build
// programs and row codes (host side of Cussen PC-MM).
#include "plan.hpp"

#include "../../include/pcmm_diag.h"

#include <algorithm>
#include <array>
#include <atomic>
#include <thread>
#include <unordered_map>

namespace pcmm {

namespace {

inline int16_t base_operand(int t) { return (int16_t)(-1 - t); }

// Compression and reconstruction schedule of one column (Alg. 2 with N
// rounds).  `vals` are |a_ik| >= 0.  Emits ops into `ops` (registers numbered
// from *nreg) and returns, for every row, the operand holding |a_ik| B_t
// (or INT16_MIN for a zero entry).
struct column_result {
    std::vector<int16_t> row_operand;  // per row
    std::vector<int16_t> level1;       // operand of each distinct nonzero value, ascending
    std::vector<int> row_rank;         // per row: rank of |a| among them, -1 for zero
    int64_t nN = 0, adds_counted = 0;
};

// Sorted distinct nonzero values of v (v >= 0) into uniq, and for each
// element of v its index among them (-1 for 0) into rank_of.  Values below
// 256 (at most 8-bit entries and their differences) use a presence table
// scanned in order; wider ones sort.
void distinct_ranks(const std::vector<int> &v, std::vector<int> &uniq, std::vector<int> &rank_of) {
    uniq.clear();
    rank_of.resize(v.size());
    int vmax = 0;
    for (int x : v) vmax = std::max(vmax, x);
    if (vmax < 256) {
        bool present[256] = {false};
        int rank[256];
        for (int x : v) present[x] = true;
        present[0] = false;  // zeros are dropped: 0 * B needs no operation
        for (int x = 1; x <= vmax; ++x)
            if (present[x]) {
                rank[x] = (int)uniq.size();
                uniq.push_back(x);
            }
        for (size_t i = 0; i < v.size(); ++i) rank_of[i] = v[i] == 0 ? -1 : rank[v[i]];
        return;
    }
    for (int x : v)
        if (x != 0) uniq.push_back(x);
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    for (size_t i = 0; i < v.size(); ++i)
        rank_of[i] = v[i] == 0 ? -1 : (int)(std::lower_bound(uniq.begin(), uniq.end(), v[i]) - uniq.begin());
}

column_result compress_column(const std::vector<int> &vals, int N, int t, std::vector<plan_op> &ops,
                              int *nreg, int64_t *mul_bits) {
    // "sort and eliminate duplicates" gives each level's distinct values; the
    // tracking pointer of a value is its rank among them
    const int m = (int)vals.size();
    column_result res;
    res.row_operand.assign(m, INT16_MIN);
    std::vector<std::vector<int>> level(N + 1);
    std::vector<int> row_rank;
    distinct_ranks(vals, level[1], row_rank);
    // ptr[w][i] for w >= 2: rank in level w of element i of level w-1
    std::vector<std::vector<int>> ptr(N + 1);
    for (int w = 1; w <= N; ++w) {
        if (w >= 2) distinct_ranks(level[w - 1], level[w], ptr[w]);
        if (w != N) {
            std::vector<int> &u = level[w];
            for (int i = (int)u.size() - 1; i >= 1; --i) u[i] -= u[i - 1];
        }
    }
    res.nN = (int64_t)level[N].size();
    for (int w = 1; w < N; ++w) res.adds_counted += (int64_t)level[w].size();
    // reconstruction: operands of level N, then prefix sums down to level 1
    std::vector<int16_t> cur(level[N].size());
    for (size_t i = 0; i < level[N].size(); ++i) {
        int s = level[N][i];
        if (s == 1) {
            cur[i] = base_operand(t);
        } else {
            plan_op op{};
            op.kind = OP_MUL;
            op.dst = (int16_t)(*nreg)++;
            op.a = base_operand(t);
            op.s = s;
            int bitsn = 0;
            while ((s >> bitsn) != 0) ++bitsn;
            *mul_bits += bitsn;
            ops.push_back(op);
            cur[i] = op.dst;
        }
    }
    for (int w = N - 1; w >= 1; --w) {
        // un-sort: element i of level w takes the operand of its difference
        std::vector<int16_t> b(level[w].size());
        for (size_t i = 0; i < level[w].size(); ++i) b[i] = cur[ptr[w + 1][i]];
        // prefix sums: S_0 = b_0, S_i = S_{i-1} + b_i
        std::vector<int16_t> S(b.size());
        for (size_t i = 0; i < b.size(); ++i) {
            if (i == 0) {
                S[i] = b[i];
            } else {
                plan_op op{};
                op.kind = OP_ADD;
                op.dst = (int16_t)(*nreg)++;
                op.a = S[i - 1];
                op.b = b[i];
                ops.push_back(op);
                S[i] = op.dst;
            }
        }
        cur = std::move(S);
    }
    // un-sort level 1 back to the rows
    for (int i = 0; i < m; ++i)
        if (row_rank[i] >= 0) res.row_operand[i] = cur[row_rank[i]];
    res.level1 = std::move(cur);
    res.row_rank = std::move(row_rank);
    return res;
}

}  // namespace

namespace {

// One column group's share of the plan: its program, its table entries and
// (written in place) its row codes.
struct group_plan {
    std::vector<plan_op> ops;
    std::vector<int16_t> entries;
    int nreg = 0;
    int64_t level_mults = 0, level_adds = 0, mul_bits = 0, accum_adds = 0;
    int err = 0;  // 0, -1 (too many registers or entries), -2 (entry outside the bit-width)
};

// Per-thread scratch: direct-mapped lookup of row segments (g <= 2, entries
// up to 8 bits), stamped with the group so it needs no clearing.
struct group_scratch {
    std::vector<int> stamp, slot, vals;
    std::vector<int32_t> col[4];
};

// The table build folds each entry's Z into its batched inversion as soon as
// the op producing the entry ends, so a group's entries must be in the order
// of their producing ops (entries that are base points, which need no
// inversion, may sit anywhere).  Reorders the entries stably by that op and
// renumbers the group's row codes to match.
void order_entries(group_plan &gp, int16_t *codes, int m) {
    const size_t E = gp.entries.size();
    std::vector<int> made_by(std::max(gp.nreg, 1), -1);
    for (size_t o = 0; o < gp.ops.size(); ++o) made_by[gp.ops[o].dst] = (int)o;
    auto key = [&](size_t e) { return gp.entries[e] < 0 ? -1 : made_by[gp.entries[e]]; };
    // already in order (always for single columns): the producing ops of the
    // register entries increase
    bool sorted = true;
    int last = -1;
    for (size_t e = 0; e < E && sorted; ++e) {
        if (key(e) < 0) continue;
        sorted = key(e) > last;
        last = key(e);
    }
    if (sorted) return;
    std::vector<int> order(E);
    for (size_t e = 0; e < E; ++e) order[e] = (int)e;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return key(x) < key(y); });
    std::vector<int16_t> entries(E);
    std::vector<int> renum(E);
    for (size_t k = 0; k < E; ++k) {
        entries[k] = gp.entries[order[k]];
        renum[order[k]] = (int)k;
    }
    gp.entries = std::move(entries);
    for (int i = 0; i < m; ++i) {
        const int c = codes[i];
        if (c != 0) codes[i] = (int16_t)(c < 0 ? -(renum[-c - 1] + 1) : renum[c - 1] + 1);
    }
}

void build_group(const void *A, int m, int n, int bits, bool is_signed, int N, int g, int key_bits, int grp,
                 int16_t *codes, group_plan &gp, group_scratch &sc) {
    const int lo = is_signed ? -(1 << (bits - 1)) : 0;
    const int hi = is_signed ? (1 << (bits - 1)) - 1 : (1 << bits) - 1;
    const int k0 = grp * g;
    const int gg = std::min(g, n - k0);
    // the group's columns of A, validated against the declared bit-width
    for (int t = 0; t < gg; ++t) {
        sc.col[t].resize(m);
        for (int i = 0; i < m; ++i) {
            const int v = plain_at(A, (int64_t)i * n + k0 + t, bits, is_signed);
            if (v < lo || v > hi) {
                gp.err = -2;
                return;
            }
            sc.col[t][i] = v;
        }
    }
    int nreg = 0;
    // per-digit tables
    std::vector<std::vector<int16_t>> digit_operand(gg);
    sc.vals.resize(m);
    for (int t = 0; t < gg; ++t) {
        const int32_t *col = sc.col[t].data();
        for (int i = 0; i < m; ++i) sc.vals[i] = std::abs((int)col[i]);
        column_result cr = compress_column(sc.vals, N, t, gp.ops, &nreg, &gp.mul_bits);
        gp.level_mults += cr.nN;
        gp.level_adds += cr.adds_counted;
        if (gg == 1) {
            // one column: the table is the level-1 reconstruction itself,
            // entry e = the e-th smallest distinct |a|; code = sign (e + 1)
            for (int i = 0; i < m; ++i) {
                if (cr.row_rank[i] < 0) continue;
                codes[i] = (int16_t)(col[i] < 0 ? -(cr.row_rank[i] + 1) : cr.row_rank[i] + 1);
                ++gp.accum_adds;
            }
            gp.entries = std::move(cr.level1);
            gp.nreg = nreg;
            if (nreg > 32000) gp.err = -1;
            else order_entries(gp, codes, m);
            return;
        }
        digit_operand[t] = std::move(cr.row_operand);
    }
    // distinct row segments up to sign (first nonzero digit made positive);
    // a segment is keyed by its digits, key_bits each
    const bool direct = gg <= 2 && key_bits == 9;
    if (direct && sc.stamp.empty()) {
        sc.stamp.assign((size_t)1 << 18, -1);
        sc.slot.assign((size_t)1 << 18, 0);
    }
    std::unordered_map<uint64_t, int> entry_of;
    for (int i = 0; i < m; ++i) {
        int seg[4] = {0, 0, 0, 0};
        int first = -1;
        for (int t = 0; t < gg; ++t) {
            seg[t] = sc.col[t][i];
            if (first < 0 && seg[t] != 0) first = t;
        }
        if (first < 0) continue;  // code 0: all-zero segment
        int sigma = seg[first] < 0 ? -1 : 1;
        uint64_t key = 0;
        for (int t = 0; t < gg; ++t) {
            seg[t] *= sigma;
            key |= (uint64_t)(seg[t] + (1 << (key_bits - 1))) << (key_bits * t);
        }
        int e = -1;
        if (direct) {
            if (sc.stamp[key] == grp) e = sc.slot[key];
        } else {
            auto it = entry_of.find(key);
            if (it != entry_of.end()) e = it->second;
        }
        if (e < 0) {
            // entry = sum_t seg_t B_t from the digit tables
            int16_t acc = INT16_MIN;
            for (int t = 0; t < gg; ++t) {
                if (seg[t] == 0) continue;
                int16_t d = digit_operand[t][i];
                if (acc == INT16_MIN) {
                    acc = d;  // first nonzero digit is positive
                } else {
                    plan_op op{};
                    op.kind = OP_ADD;
                    op.dst = (int16_t)nreg++;
                    op.a = acc;
                    op.b = d;
                    op.neg_b = seg[t] < 0 ? 1 : 0;
                    gp.ops.push_back(op);
                    acc = op.dst;
                }
            }
            e = (int)gp.entries.size();
            gp.entries.push_back(acc);
            if (direct) {
                sc.stamp[key] = grp;
                sc.slot[key] = e;
            } else {
                entry_of.emplace(key, e);
            }
        }
        codes[i] = (int16_t)(sigma * (e + 1));
        ++gp.accum_adds;
    }
    gp.nreg = nreg;
    if (nreg > 32000 || gp.entries.size() > 32000) gp.err = -1;
    else order_entries(gp, codes, m);
}

}  // namespace

int build_cussen_plan(const void *A, int m, int n, int bits, bool is_signed, int N, int g, cussen_plan *out,
                      int threads) {
    if (!out || m < 0 || n < 0 || bits < 1 || bits > 16 || N < 1 || N > 8 || g < 1 || g > 4) return -1;
    if ((int64_t)m * n > 0 && !A) return -1;
    if (m > 32767) return -1;
    // row segments of g digits are keyed with 9 bits per digit up to 8-bit
    // entries and 17 bits beyond (so at most 3 digits fit the 64-bit key)
    const int key_bits = bits <= 8 ? 9 : 17;
    if (g * key_bits > 64) return -1;
    cussen_plan P;
    P.m = m;
    P.n = n;
    P.g = g;
    P.N = N;
    P.ngroups = (n + g - 1) / g;
    P.codes.assign((size_t)P.ngroups * m, 0);
    // the groups are independent: built on up to `threads` threads (at least
    // 16 groups each), then concatenated in group order
    std::vector<group_plan> parts(P.ngroups);
    const int nthreads = std::max(1, std::min(threads, P.ngroups / 16));
    std::atomic<int> next{0};
    auto worker = [&]() {
        group_scratch sc;
        for (int grp = next++; grp < P.ngroups; grp = next++)
            build_group(A, m, n, bits, is_signed, N, g, key_bits, grp, &P.codes[(size_t)grp * m], parts[grp], sc);
    };
    if (nthreads <= 1) {
        worker();
    } else {
        std::vector<std::thread> pool;
        for (int t = 0; t < nthreads; ++t) pool.emplace_back(worker);
        for (auto &th : pool) th.join();
    }
    for (const group_plan &gp : parts)
        if (gp.err == -2) return -2;
    for (const group_plan &gp : parts)
        if (gp.err) return gp.err;
    size_t nops = 0, nent = 0;
    for (const group_plan &gp : parts) {
        nops += gp.ops.size();
        nent += gp.entries.size();
    }
    P.ops.reserve(nops);
    P.entries.reserve(nent);
    P.op_begin.reserve(P.ngroups + 1);
    P.entry_begin.reserve(P.ngroups + 1);
    P.op_begin.push_back(0);
    P.entry_begin.push_back(0);
    for (group_plan &gp : parts) {
        P.ops.insert(P.ops.end(), gp.ops.begin(), gp.ops.end());
        P.entries.insert(P.entries.end(), gp.entries.begin(), gp.entries.end());
        P.op_begin.push_back((int32_t)P.ops.size());
        P.entry_begin.push_back((int32_t)P.entries.size());
        P.nregs.push_back(gp.nreg);
        P.max_regs = std::max(P.max_regs, gp.nreg);
        P.max_entries = std::max(P.max_entries, (int)gp.entries.size());
        P.table_entries += (int64_t)gp.entries.size();
        P.level_mults += gp.level_mults;
        P.level_adds += gp.level_adds;
        P.table_mul_bits += gp.mul_bits;
        P.accum_adds += gp.accum_adds;
    }
    for (const plan_op &op : P.ops)
        if (op.kind == OP_ADD) ++P.table_adds;
    *out = std::move(P);
    return 0;
}

// Verifies a plan by running every group's program on integer coefficient
// vectors over the group's base points (B_t -> the t-th unit vector).  0 when
// the plan is sound, else the first failure: 1 register entries out of the
// order of their producing ops, 2 a code outside its group's table, 3 an
// entry that is not the row segment its code stands for, 4 a malformed
// program (operand undefined or out of range, a register written twice).
int check_cussen_plan(const cussen_plan &P, const void *A, int bits, bool is_signed) {
    const int m = P.m, n = P.n, g = P.g;
    if ((int)P.op_begin.size() != P.ngroups + 1 || (int)P.entry_begin.size() != P.ngroups + 1 ||
        (int)P.nregs.size() != P.ngroups || P.codes.size() != (size_t)P.ngroups * m)
        return 4;
    using vec = std::array<int64_t, 4>;
    for (int grp = 0; grp < P.ngroups; ++grp) {
        const int k0 = grp * g;
        const int gg = std::min(g, n - k0);
        const int nreg = P.nregs[grp];
        std::vector<vec> reg(std::max(nreg, 1));
        std::vector<int> made_by(std::max(nreg, 1), -1);
        bool bad = false;
        auto value = [&](int16_t opd) -> vec {
            vec v{0, 0, 0, 0};
            if (opd < 0) {
                const int t = -1 - opd;
                if (t >= gg) bad = true;
                else v[t] = 1;
            } else if (opd >= nreg || made_by[opd] < 0) {
                bad = true;
            } else {
                v = reg[opd];
            }
            return v;
        };
        for (int o = P.op_begin[grp]; o < P.op_begin[grp + 1]; ++o) {
            const plan_op &op = P.ops[o];
            if (op.dst < 0 || op.dst >= nreg || made_by[op.dst] >= 0) return 4;
            vec r{0, 0, 0, 0};
            if (op.kind == OP_MUL) {
                if (op.a >= 0 || op.s < 1) return 4;
                const vec b = value(op.a);
                for (int t = 0; t < 4; ++t) r[t] = (int64_t)op.s * b[t];
            } else if (op.kind == OP_ADD) {
                const vec x = value(op.a), y = value(op.b);
                for (int t = 0; t < 4; ++t) r[t] = x[t] + (op.neg_b ? -y[t] : y[t]);
            } else {
                return 4;
            }
            if (bad) return 4;
            reg[op.dst] = r;
            made_by[op.dst] = o;
        }
        const int eb = P.entry_begin[grp], E = P.entry_begin[grp + 1] - eb;
        std::vector<vec> ent(E);
        int last = -1;
        for (int e = 0; e < E; ++e) {
            const int16_t opd = P.entries[eb + e];
            ent[e] = value(opd);
            if (bad) return 4;
            if (opd >= 0) {
                if (made_by[opd] <= last) return 1;
                last = made_by[opd];
            }
        }
        for (int i = 0; i < m; ++i) {
            vec seg{0, 0, 0, 0};
            bool zero = true;
            for (int t = 0; t < gg; ++t) {
                seg[t] = plain_at(A, (int64_t)i * n + k0 + t, bits, is_signed);
                zero = zero && seg[t] == 0;
            }
            const int c = P.codes[(size_t)grp * m + i];
            if (zero != (c == 0)) return 3;
            if (c == 0) continue;
            const int e = (c < 0 ? -c : c) - 1;
            if (e >= E) return 2;
            for (int t = 0; t < 4; ++t)
                if ((c < 0 ? -ent[e][t] : ent[e][t]) != seg[t]) return 3;
        }
    }
    return 0;
}

}  // namespace pcmm

extern "C" pcmm_status pcmm_diag_plan_check(const void *A, int32_t m, int32_t n, int32_t bits, int32_t is_signed,
                                            int32_t rounds, int32_t group, int32_t *result) {
    if (!result || m < 0 || n < 0 || bits < 1 || bits > 16 || rounds < 1 || rounds > 8 || group < 1 || group > 4)
        return PCMM_EINVAL;
    pcmm::cussen_plan P;
    const int rc = pcmm::build_cussen_plan(A, m, n, bits, is_signed != 0, rounds, group, &P, 4);
    if (rc == -2) return PCMM_ERANGE;
    if (rc) return PCMM_EINVAL;
    *result = pcmm::check_cussen_plan(P, A, bits, is_signed != 0);
    return PCMM_OK;
}
