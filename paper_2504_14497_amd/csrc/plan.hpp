// plan.hpp -- host-side compression plan for Cussen PC-MM (internal).
//
// For each column group of A (g consecutive columns; g = 1 is Alg. 3 as
// printed) the plan holds
//   * a straight-line program that builds, for one output column j and one
//     ciphertext point, the table of point multiples needed by the group:
//       MUL  dst = s * B_t                      (Alg. 2 level-N multiply, Alg. 1)
//       ADD  dst = src_a + (-1)^neg * src_b     (Alg. 2 prefix sums; for g > 1 also
//                                               the combination of the g digits)
//     where an operand is a register (the result of an earlier op) or one of
//     the group's base points B_t = B[k0 + t, j] (affine input);
//   * the table entries, each an operand of that program;
//   * one code per row: 0 for an all-zero row segment, else +-(entry + 1).
// The un-sort / re-insert steps of the reconstruction are resolved at plan
// time into operand references, so the GPU executes only point operations.
#pragma once
#include <stdint.h>

#include <vector>

namespace pcmm {

enum : uint8_t { OP_MUL = 1, OP_ADD = 2 };

// operand: >= 0 register id; < 0 base point t = -1 - operand
struct plan_op {
    uint8_t kind;
    uint8_t neg_b;  // ADD: subtract operand b
    int16_t dst;
    int16_t a;      // ADD: first operand; MUL: base index operand (< 0)
    int16_t b;      // ADD: second operand
    int32_t s;      // MUL: small non-negative scalar
};

struct cussen_plan {
    int m = 0, n = 0, g = 1, N = 4, ngroups = 0;
    int max_entries = 0;   // E: largest table of a group (layout stride)
    int max_regs = 0;      // largest register count of a group
    std::vector<int32_t> op_begin;      // ngroups + 1
    std::vector<plan_op> ops;
    std::vector<int32_t> nregs;         // per group
    std::vector<int32_t> entry_begin;   // ngroups + 1
    std::vector<int16_t> entries;       // operand of every table entry
    std::vector<int16_t> codes;         // ngroups x m (group-major)
    // operation counts
    int64_t level_mults = 0;   // sum over columns of n_N
    int64_t level_adds = 0;    // sum over columns of sum_{w<N} n_w (paper's counting)
    int64_t table_adds = 0;    // ADD ops per (output column, point)
    int64_t table_mul_bits = 0;  // sum of ladder lengths of MUL ops
    int64_t accum_adds = 0;    // nonzero codes (mixed additions per output column and point)
    int64_t table_entries = 0;
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
