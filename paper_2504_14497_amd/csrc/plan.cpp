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
    std::vector<int32_t> level1_values;  // those values
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
    res.level1_values.assign(level[1].begin(), level[1].end());
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

// One column of a group: its digit-table program and entries.
struct unit_plan {
    std::vector<plan_op> ops;
    std::vector<int16_t> entries;  // level-1 operands, ascending values
    std::vector<int32_t> values;   // the value (multiple of the base point) of each entry
    std::vector<int> pos_of_rank;  // rank of a value among them -> position in `entries`
    int nreg = 0;
};

// One column group's share of the plan: its units, its combinations and
// (written in place) its row codes.
struct group_plan {
    std::vector<unit_plan> units;
    std::vector<plan_combo> combos;
    std::vector<plan_cblock> cblocks;  // run indices local to the group
    std::vector<plan_crun> cruns;
    int entries = 0;  // entries of the group's table
    int levels = 1;
    int64_t level_mults = 0, level_adds = 0, mul_bits = 0, accum_adds = 0;
    int err = 0;  // 0, -1 (too many registers or entries), -2 (entry outside the bit-width)
};

// Per-thread scratch: direct-mapped lookup of row segments (g <= 2, entries
// up to 8 bits; bits + 1 bits per digit, so 2^(2 bits + 2) slots), stamped
// with the group so it needs no clearing.
struct group_scratch {
    std::vector<int> stamp, slot, vals;
    std::vector<int32_t> col[4];
};

// The digit-table build folds each entry's Z into its batched inversion as
// soon as the op producing the entry ends, so a unit's entries must be in
// the order of their producing ops (entries that are the base point, which
// need no inversion, may sit anywhere).  Reorders the entries stably by that
// op and records where each rank went.
void order_entries(unit_plan &u) {
    const size_t E = u.entries.size();
    u.pos_of_rank.resize(E);
    for (size_t e = 0; e < E; ++e) u.pos_of_rank[e] = (int)e;
    std::vector<int> made_by(std::max(u.nreg, 1), -1);
    for (size_t o = 0; o < u.ops.size(); ++o) made_by[u.ops[o].dst] = (int)o;
    auto key = [&](size_t e) { return u.entries[e] < 0 ? -1 : made_by[u.entries[e]]; };
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
    std::vector<int32_t> values(E);
    for (size_t k = 0; k < E; ++k) {
        entries[k] = u.entries[order[k]];
        values[k] = u.values[order[k]];
        u.pos_of_rank[order[k]] = (int)k;
    }
    u.entries = std::move(entries);
    u.values = std::move(values);
}

void block_combos(group_plan &gp);

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
    // digit tables: Alg. 2 on each column's magnitudes
    gp.units.assign(gg, unit_plan{});
    std::vector<std::vector<int>> rank(gg);
    std::vector<int> off(gg, 0);
    sc.vals.resize(m);
    int entries = 0;
    for (int t = 0; t < gg; ++t) {
        unit_plan &u = gp.units[t];
        const int32_t *col = sc.col[t].data();
        for (int i = 0; i < m; ++i) sc.vals[i] = std::abs((int)col[i]);
        column_result cr = compress_column(sc.vals, N, 0, u.ops, &u.nreg, &gp.mul_bits);
        gp.level_mults += cr.nN;
        gp.level_adds += cr.adds_counted;
        u.entries = std::move(cr.level1);
        u.values = std::move(cr.level1_values);
        if (u.nreg > 32000) {
            gp.err = -1;
            return;
        }
        order_entries(u);
        rank[t] = std::move(cr.row_rank);
        off[t] = entries;
        entries += (int)u.entries.size();
    }
    auto digit_entry = [&](int t, int i) { return off[t] + gp.units[t].pos_of_rank[rank[t][i]]; };
    if (gg == 1) {
        // one column: the table is the level-1 reconstruction itself; code =
        // sign (entry + 1)
        const int32_t *col = sc.col[0].data();
        for (int i = 0; i < m; ++i) {
            if (rank[0][i] < 0) continue;
            const int e = digit_entry(0, i);
            codes[i] = (int16_t)(col[i] < 0 ? -(e + 1) : e + 1);
            ++gp.accum_adds;
        }
        gp.entries = entries;
        return;
    }
    // Row segments up to sign (first nonzero digit made positive).  A
    // segment's entry is built digit by digit: the entry of its prefix
    // (s_0 .. s_{t-1}) plus s_t times digit t's entry, one combination per
    // distinct prefix with at least two nonzero digits (memoised on the
    // prefix, keyed by its digits, key_bits each, and its length).
    const bool direct = gg <= 2 && key_bits == 9;
    const int dbits = bits + 1;  // digit + 2^bits lies in [0, 2^(bits+1))
    if (direct && sc.stamp.empty()) {
        sc.stamp.assign((size_t)1 << (2 * dbits), -1);
        sc.slot.assign((size_t)1 << (2 * dbits), 0);
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
        const int sigma = seg[first] < 0 ? -1 : 1;
        int cur = -1, nz = 0;
        uint64_t key = 0, dkey = 0;
        for (int t = 0; t < gg; ++t) {
            seg[t] *= sigma;
            key |= (uint64_t)(seg[t] + (1 << (key_bits - 1))) << (key_bits * t);
            dkey |= (uint64_t)(seg[t] + (1 << bits)) << (dbits * t);
            if (seg[t] == 0) continue;
            const int d = digit_entry(t, i);
            ++nz;
            if (cur < 0) {  // the first nonzero digit (positive)
                cur = d;
                continue;
            }
            // the prefix up to t: its digits and its length
            const uint64_t pkey = key | ((uint64_t)t << 62);
            int e = -1;
            if (direct) {
                if (sc.stamp[dkey] == grp) e = sc.slot[dkey];
            } else {
                auto it = entry_of.find(pkey);
                if (it != entry_of.end()) e = it->second;
            }
            if (e < 0) {
                e = entries++;
                plan_combo c{};
                c.dst = (int16_t)e;
                c.a = (int16_t)cur;
                c.b = (int16_t)d;
                c.neg_b = seg[t] < 0 ? 1 : 0;
                c.level = (uint8_t)nz;
                gp.combos.push_back(c);
                gp.levels = std::max(gp.levels, nz);
                if (direct) {
                    sc.stamp[dkey] = grp;
                    sc.slot[dkey] = e;
                } else {
                    entry_of.emplace(pkey, e);
                }
            }
            cur = e;
        }
        codes[i] = (int16_t)(sigma * (cur + 1));
        ++gp.accum_adds;
    }
    gp.entries = entries;
    if (entries > 32000) {
        gp.err = -1;
        return;
    }
    // one level after another (a combination's first operand has the level
    // below its own, its second is a digit entry); within a level by first
    // operand, so the GPU keeps it in registers over a run of combinations
    std::sort(gp.combos.begin(), gp.combos.end(), [](const plan_combo &x, const plan_combo &y) {
        if (x.level != y.level) return x.level < y.level;
        if (x.a != y.a) return x.a < y.a;
        return x.b < y.b;
    });
    block_combos(gp);
}

// Blocks of up to COMBO_BLOCK consecutive first operands per level, each
// with its runs by second operand (ascending).
void block_combos(group_plan &gp) {
    const auto &C = gp.combos;
    size_t c = 0;
    while (c < C.size()) {
        plan_cblock blk{};
        blk.level = C[c].level;
        blk.run_begin = (int32_t)gp.cruns.size();
        size_t e = c;  // combinations of the block: [c, e)
        while (e < C.size() && C[e].level == blk.level) {
            if (e == c || C[e].a != C[e - 1].a) {
                if (blk.na == COMBO_BLOCK) break;
                blk.a[blk.na++] = C[e].a;
            }
            ++e;
        }
        // runs by second operand; a + b and a - b (signed plaintexts) both
        // occur, so a run ends where its slot for a combination's a is taken
        std::vector<size_t> idx;
        for (size_t k = c; k < e; ++k) idx.push_back(k);
        std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
            return C[x].b != C[y].b ? C[x].b < C[y].b : C[x].neg_b < C[y].neg_b;
        });
        for (size_t k = 0; k < idx.size();) {
            plan_crun run{};
            run.b = C[idx[k]].b;
            for (int r = 0; r < COMBO_BLOCK; ++r) run.dst[r] = -1;
            for (; k < idx.size() && C[idx[k]].b == run.b; ++k) {
                const plan_combo &cm = C[idx[k]];
                int r = 0;
                while (blk.a[r] != cm.a) ++r;
                if (run.dst[r] >= 0) break;
                run.dst[r] = cm.dst;
                if (cm.neg_b) run.neg |= (uint8_t)(1u << r);
            }
            gp.cruns.push_back(run);
        }
        blk.run_end = (int32_t)gp.cruns.size();
        gp.cblocks.push_back(blk);
        c = e;
    }
}

}  // namespace

int build_cussen_plan(const void *A, int m, int n, int bits, bool is_signed, int N, int g, cussen_plan *out,
                      int threads) {
    if (!out || m < 0 || n < 0 || bits < 1 || bits > 16 || N < 1 || N > 8 || g < 1 || g > 4) return -1;
    if ((int64_t)m * n > 0 && !A) return -1;
    if (m > 32767) return -1;
    // row segments of g digits are keyed with 9 bits per digit up to 8-bit
    // entries and 17 bits beyond (so at most 3 digits fit beside the length)
    const int key_bits = bits <= 8 ? 9 : 17;
    if (g * key_bits > 62) return -1;
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
    size_t nops = 0, nent = 0, ncombo = 0;
    for (const group_plan &gp : parts) {
        for (const unit_plan &u : gp.units) {
            nops += u.ops.size();
            nent += u.entries.size();
        }
        ncombo += gp.combos.size();
    }
    P.ops.reserve(nops);
    P.entries.reserve(nent);
    P.entry_value.reserve(nent);
    P.combos.reserve(ncombo);
    P.op_begin.push_back(0);
    P.entry_begin.push_back(0);
    P.combo_begin.push_back(0);
    P.cblock_begin.push_back(0);
    for (int grp = 0; grp < P.ngroups; ++grp) {
        group_plan &gp = parts[grp];
        int off = 0;
        for (size_t t = 0; t < gp.units.size(); ++t) {
            unit_plan &u = gp.units[t];
            P.unit_col.push_back(grp * g + (int)t);
            P.unit_grp.push_back(grp);
            P.unit_off.push_back(off);
            off += (int)u.entries.size();
            P.ops.insert(P.ops.end(), u.ops.begin(), u.ops.end());
            P.entries.insert(P.entries.end(), u.entries.begin(), u.entries.end());
            P.entry_value.insert(P.entry_value.end(), u.values.begin(), u.values.end());
            P.op_begin.push_back((int32_t)P.ops.size());
            P.entry_begin.push_back((int32_t)P.entries.size());
            P.nregs.push_back(u.nreg);
            P.max_regs = std::max(P.max_regs, u.nreg);
            P.digit_entries += (int64_t)u.entries.size();
        }
        P.combos.insert(P.combos.end(), gp.combos.begin(), gp.combos.end());
        P.combo_begin.push_back((int32_t)P.combos.size());
        const int32_t run0 = (int32_t)P.cruns.size();
        for (plan_cblock blk : gp.cblocks) {
            blk.run_begin += run0;
            blk.run_end += run0;
            P.cblocks.push_back(blk);
        }
        P.cruns.insert(P.cruns.end(), gp.cruns.begin(), gp.cruns.end());
        P.cblock_begin.push_back((int32_t)P.cblocks.size());
        P.group_entries.push_back(gp.entries);
        P.max_entries = std::max(P.max_entries, gp.entries);
        P.max_levels = std::max(P.max_levels, gp.levels);
        P.table_entries += gp.entries;
        P.level_mults += gp.level_mults;
        P.level_adds += gp.level_adds;
        P.table_mul_bits += gp.mul_bits;
        P.accum_adds += gp.accum_adds;
    }
    P.nunits = (int)P.unit_col.size();
    for (const plan_op &op : P.ops)
        if (op.kind == OP_ADD) ++P.table_adds;
    P.combo_adds = (int64_t)P.combos.size();
    P.table_adds += P.combo_adds;
    *out = std::move(P);
    return 0;
}

// Verifies a plan by running every unit's program and every group's
// combinations on integer coefficient vectors over the group's base points
// (B_t -> the t-th unit vector).  0 when the plan is sound, else the first
// failure: 1 digit entries out of the order of their producing ops, 2 a code
// outside its group's table, 3 an entry that is not the row segment its code
// stands for, 4 a malformed program (an operand undefined or out of range, a
// register or entry written twice, a unit outside its group, a combination
// reading a level not below its own).
int check_cussen_plan(const cussen_plan &P, const void *A, int bits, bool is_signed) {
    const int m = P.m, n = P.n, g = P.g;
    if ((int)P.op_begin.size() != P.nunits + 1 || (int)P.entry_begin.size() != P.nunits + 1 ||
        P.entry_value.size() != P.entries.size() ||
        (int)P.nregs.size() != P.nunits || (int)P.unit_col.size() != P.nunits ||
        (int)P.unit_grp.size() != P.nunits || (int)P.unit_off.size() != P.nunits ||
        (int)P.combo_begin.size() != P.ngroups + 1 || (int)P.cblock_begin.size() != P.ngroups + 1 ||
        (int)P.group_entries.size() != P.ngroups ||
        P.codes.size() != (size_t)P.ngroups * m)
        return 4;
    using vec = std::array<int64_t, 4>;
    int u = 0;
    for (int grp = 0; grp < P.ngroups; ++grp) {
        const int k0 = grp * g;
        const int gg = std::min(g, n - k0);
        const int E = P.group_entries[grp];
        if (E < 0 || E > P.max_entries) return 4;
        std::vector<vec> ent(E, vec{0, 0, 0, 0});
        std::vector<int> level(E, 0);  // 0: not yet defined
        // the group's units: digit t of the group is column k0 + t
        for (int t = 0; t < gg; ++t, ++u) {
            if (u >= P.nunits || P.unit_grp[u] != grp || P.unit_col[u] != k0 + t) return 4;
            const int nreg = P.nregs[u];
            std::vector<vec> reg(std::max(nreg, 1));
            std::vector<int> made_by(std::max(nreg, 1), -1);
            bool bad = false;
            auto value = [&](int16_t opd) -> vec {
                vec v{0, 0, 0, 0};
                if (opd < 0) {
                    if (opd != -1) bad = true;
                    else v[t] = 1;
                } else if (opd >= nreg || made_by[opd] < 0) {
                    bad = true;
                } else {
                    v = reg[opd];
                }
                return v;
            };
            for (int o = P.op_begin[u]; o < P.op_begin[u + 1]; ++o) {
                const plan_op &op = P.ops[o];
                if (op.dst < 0 || op.dst >= nreg || made_by[op.dst] >= 0) return 4;
                vec r{0, 0, 0, 0};
                if (op.kind == OP_MUL) {
                    if (op.a >= 0 || op.s < 1) return 4;
                    const vec b = value(op.a);
                    for (int q = 0; q < 4; ++q) r[q] = (int64_t)op.s * b[q];
                } else if (op.kind == OP_ADD) {
                    const vec x = value(op.a), y = value(op.b);
                    for (int q = 0; q < 4; ++q) r[q] = x[q] + (op.neg_b ? -y[q] : y[q]);
                } else {
                    return 4;
                }
                if (bad) return 4;
                reg[op.dst] = r;
                made_by[op.dst] = o;
            }
            const int eb = P.entry_begin[u], ne = P.entry_begin[u + 1] - eb;
            const int off = P.unit_off[u];
            if (off < 0 || off + ne > E) return 4;
            int last = -1;
            for (int e = 0; e < ne; ++e) {
                const int16_t opd = P.entries[eb + e];
                if (level[off + e]) return 4;
                ent[off + e] = value(opd);
                // the recorded value: this multiple of digit t's base point
                for (int q = 0; q < 4; ++q)
                    if (ent[off + e][q] != (q == t ? (int64_t)P.entry_value[eb + e] : 0)) return 3;
                level[off + e] = 1;
                if (bad) return 4;
                if (opd >= 0) {
                    if (made_by[opd] <= last) return 1;
                    last = made_by[opd];
                }
            }
        }
        for (int c = P.combo_begin[grp]; c < P.combo_begin[grp + 1]; ++c) {
            const plan_combo &cb = P.combos[c];
            if (cb.dst < 0 || cb.dst >= E || cb.a < 0 || cb.a >= E || cb.b < 0 || cb.b >= E) return 4;
            if (level[cb.dst] || !level[cb.a] || level[cb.b] != 1 || level[cb.a] >= cb.level) return 4;
            if (c > P.combo_begin[grp] && P.combos[c - 1].level > cb.level) return 4;
            for (int q = 0; q < 4; ++q) ent[cb.dst][q] = ent[cb.a][q] + (cb.neg_b ? -ent[cb.b][q] : ent[cb.b][q]);
            level[cb.dst] = cb.level;
        }
        for (int e = 0; e < E; ++e)
            if (!level[e]) return 4;
        // the blocked form holds exactly the group's combinations
        {
            std::vector<int> seen(E, 0);
            size_t count = 0;
            int last_level = 0;
            for (int bi = P.cblock_begin[grp]; bi < P.cblock_begin[grp + 1]; ++bi) {
                const plan_cblock &blk = P.cblocks[bi];
                if (blk.na < 1 || blk.na > COMBO_BLOCK || blk.level < last_level) return 4;
                last_level = blk.level;
                for (int ri = blk.run_begin; ri < blk.run_end; ++ri) {
                    const plan_crun &run = P.cruns[ri];
                    for (int r = 0; r < COMBO_BLOCK; ++r) {
                        if (run.dst[r] < 0) continue;
                        if (r >= blk.na || run.dst[r] >= E || seen[run.dst[r]]++) return 4;
                        bool found = false;
                        for (int c = P.combo_begin[grp]; c < P.combo_begin[grp + 1] && !found; ++c) {
                            const plan_combo &cb = P.combos[c];
                            found = cb.dst == run.dst[r] && cb.a == blk.a[r] && cb.b == run.b &&
                                    cb.neg_b == ((run.neg >> r) & 1) && cb.level == blk.level;
                        }
                        if (!found) return 4;
                        ++count;
                    }
                }
            }
            if (count != (size_t)(P.combo_begin[grp + 1] - P.combo_begin[grp])) return 4;
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
            for (int q = 0; q < 4; ++q)
                if ((c < 0 ? -ent[e][q] : ent[e][q]) != seg[q]) return 3;
        }
    }
    return u == P.nunits ? 0 : 4;
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
