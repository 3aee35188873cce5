// plan.hpp -- host-side compression plan for Cussen PC-MM (internal).
//
// A column group is g consecutive columns of A (g = 1 is Alg. 3 as printed).
// Its table, for one output column j and one ciphertext point, holds every
// point the group's rows need: first each column's digit table (Alg. 2
// reconstruction of that column), then the combinations of digits that the
// group's row segments use.  The plan holds
//   * per column ("unit") a straight-line program that builds the column's
//     digit table from its base point B_k = B[k, j]:
//       MUL  dst = s * B_k                      (Alg. 2 level-N multiply, Alg. 1)
//       ADD  dst = src_a + (-1)^neg * src_b     (Alg. 2 prefix sums)
//     where an operand is a register (the result of an earlier op of the
//     unit) or the base point itself, and the unit's level-1 entries (the
//     digit table, ascending values) as operands of that program;
//   * per group (g > 1) the combinations, each one addition of two entries
//     of the group's table, dst = a + (-1)^neg * b, ordered by level (the
//     number of nonzero digits), so one level depends only on lower ones;
//   * one code per row: 0 for an all-zero row segment, else +-(entry + 1).
// The un-sort / re-insert steps of the reconstruction are resolved at plan
// time into operand references, so the GPU executes only point operations.
#pragma once
#include <stdint.h>

#include <vector>

namespace pcmm {

enum : uint8_t { OP_MUL = 1, OP_ADD = 2 };

// operand: >= 0 register id; < 0 the unit's base point
struct plan_op {
    uint8_t kind;
    uint8_t neg_b;  // ADD: subtract operand b
    int16_t dst;
    int16_t a;      // ADD: first operand; MUL: base point operand (< 0)
    int16_t b;      // ADD: second operand
    int32_t s;      // MUL: small non-negative scalar
};

// One combination entry of a group's table: dst = a + (-1)^neg_b b, all
// three entry indices of the group's table; level = nonzero digits of dst.
struct plan_combo {
    int16_t dst, a, b;
    uint8_t neg_b;
    uint8_t level;
};

// The same combinations blocked for register reuse: a block holds up to
// COMBO_BLOCK first operands of one level (consecutive in the sorted list)
// and runs; a run is one second operand b and the combinations a[r] +- b
// that the block's rows need (dst[r] < 0: none).
constexpr int COMBO_BLOCK = 2;

struct plan_cblock {
    int16_t a[COMBO_BLOCK];
    int32_t run_begin, run_end;
    uint8_t level, na, pad[2];
};

struct plan_crun {
    int16_t b;
    int16_t dst[COMBO_BLOCK];
    uint8_t neg;  // bit r: subtract b for a[r]
    uint8_t pad;
};

struct cussen_plan {
    int m = 0, n = 0, g = 1, N = 4, ngroups = 0, nunits = 0;
    int max_entries = 0;      // E: largest table of a group (layout stride)
    int max_regs = 0;         // largest register count of a unit
    int max_levels = 1;       // largest combination level of a group (1: none)
    std::vector<int32_t> unit_col;      // nunits: column of A (row of B) of the unit
    std::vector<int32_t> unit_grp;      // nunits: its group
    std::vector<int32_t> unit_off;      // nunits: offset of its digit table in the group's table
    std::vector<int32_t> op_begin;      // nunits + 1
    std::vector<plan_op> ops;
    std::vector<int32_t> nregs;         // per unit
    std::vector<int32_t> entry_begin;   // nunits + 1
    std::vector<int16_t> entries;       // operand of every digit-table entry
    std::vector<int32_t> entry_value;   // the multiple of its column's base point each entry is
    std::vector<int32_t> combo_begin;   // ngroups + 1
    std::vector<plan_combo> combos;
    std::vector<int32_t> cblock_begin;  // ngroups + 1
    std::vector<plan_cblock> cblocks;   // runs indexed into cruns (whole plan)
    std::vector<plan_crun> cruns;
    std::vector<int32_t> group_entries; // ngroups: entries of each group's table
    std::vector<int16_t> codes;         // ngroups x m (group-major)
    // operation counts
    int64_t level_mults = 0;   // sum over columns of n_N
    int64_t level_adds = 0;    // sum over columns of sum_{w<N} n_w (paper's counting)
    int64_t table_adds = 0;    // point additions per (output column, point): ADD ops + combinations
    int64_t combo_adds = 0;    // of which combinations
    int64_t table_mul_bits = 0;  // sum of ladder lengths of MUL ops
    int64_t accum_adds = 0;    // nonzero codes (mixed additions per output column and point)
    int64_t table_entries = 0; // entries of all groups' tables
    int64_t digit_entries = 0; // of which digit-table entries
};

// Plaintext element x of A: int8 / uint8 for bits <= 8, int16 / uint16 for
// 9..16 bits (row-major).
inline int plain_at(const void *A, int64_t x, int bits, bool is_signed) {
    if (bits <= 8) return is_signed ? (int)((const int8_t *)A)[x] : (int)((const uint8_t *)A)[x];
    return is_signed ? (int)((const int16_t *)A)[x] : (int)((const uint16_t *)A)[x];
}

// Validates A (m x n row-major, elements as plain_at reads them) against its
// declared bit-width (1..16) and builds the plan, on up to `threads` host
// threads (column groups are independent).  Returns 0, or -1 (bad
// arguments, including g > 3 with entries wider than 8 bits) / -2 (an entry
// outside the bit-width).
int build_cussen_plan(const void *A, int m, int n, int bits, bool is_signed, int N, int g, cussen_plan *out,
                      int threads = 1);

// Runs each group's program on integer coefficient vectors and checks the
// plan against A (see plan.cpp): 0 when sound, else the failed check.
int check_cussen_plan(const cussen_plan &P, const void *A, int bits, bool is_signed);

}  // namespace pcmm
