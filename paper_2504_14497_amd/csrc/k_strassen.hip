// k_strassen.hip -- PC-MM by Strassen's block recursion (Sec. 3.1) on gfx950.
//
// A (plaintext), B (ciphertexts) and C are split into 2 x 2 blocks; the seven
// block products
//   M1 = (A11 + A22)(B11 + B22)   M2 = (A21 + A22) B11   M3 = A11 (B12 - B22)
//   M4 = A22 (B21 - B11)          M5 = (A11 + A12) B22   M6 = (A21 - A11)(B11 + B12)
//   M7 = (A12 - A22)(B21 + B22)
// recurse, and C11 = M1 + M4 - M5 + M7, C12 = M3 + M5, C21 = M2 + M4,
// C22 = M1 - M2 + M3 + M6.  The recursion runs breadth first to a depth D:
//   * B side, level d -> d + 1: one launch forms the seven children of every
//     node (point additions / subtractions of quadrants, Jacobian), then one
//     batched normalisation makes them affine for the next level;
//   * A side: the plaintext sums are exact integers, formed on the host
//     (their bit-width grows by at most one per level and is tracked per leaf);
//   * leaves: one launch of the schoolbook product (Alg. 1 ladders over each
//     leaf's own bit-width) for all 7^D leaf products;
//   * C side, level d + 1 -> d: one launch adds the children's outputs into the
//     four quadrants of every parent node.
// Shapes that are not multiples of 2^D are padded (zeros in A, infinity in B)
// and C is cropped.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "normalize.hpp"
#include "plan.hpp"

using namespace pcmm;

namespace {

constexpr int AFF2_PLANES = 2 * 2 * NL;  // internal affine ciphertext: 2 points x (x, y)

// quadrants (row half, column half) of the B operands of the seven children:
// child = sa * quadrant qa + sb * quadrant qb (sb = 0: a single quadrant)
struct child_b {
    int qa, sb, qb;
};
// quadrant index: 0 = 11, 1 = 12, 2 = 21, 3 = 22
__constant__ child_b CHILD_B[7] = {{0, +1, 3}, {0, 0, 0}, {1, -1, 3}, {2, -1, 0}, {3, 0, 0}, {0, +1, 1}, {2, +1, 3}};

// C quadrant q = sum over its terms of sign * M_child
struct quad_c {
    int n;
    int child[4];
    int sign[4];
};
__constant__ quad_c QUAD_C[4] = {{4, {0, 3, 4, 6}, {+1, +1, -1, +1}},
                                 {2, {2, 4, 0, 0}, {+1, +1, 0, 0}},
                                 {2, {1, 3, 0, 0}, {+1, +1, 0, 0}},
                                 {4, {0, 1, 2, 5}, {+1, -1, +1, +1}}};

// Level d -> d + 1 of the B side.  Parent level: `nodes` blocks of nb x lb
// (block q, row r, column c at element q*nb*lb + r*lb + c); at level 0 the
// parent is B itself (n0 x l0 valid, padded with infinity to nb x lb).
// Child level (Jacobian, internal): nodes*7 blocks of (nb/2) x (lb/2).
__global__ void __launch_bounds__(256) split_b_kernel(const uint32_t *__restrict__ par, int64_t ld_par,
                                                      int top, int n0, int l0, int64_t nodes, int nb, int lb,
                                                      uint32_t *__restrict__ out, int64_t ld_out) {
    const int hb = nb / 2, hl = lb / 2;
    const int64_t per_child = (int64_t)hb * hl;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = nodes * 7 * per_child * 2;
    if (t >= total) return;
    const int pt = (int)(t & 1);
    const int64_t e_out = t >> 1;  // child element
    const int64_t qc = e_out / per_child;
    const int64_t rem = e_out - qc * per_child;
    const int r = (int)(rem / hl), c = (int)(rem % hl);
    const int64_t q = qc / 7;
    const int ch = (int)(qc % 7);
    const child_b cb = CHILD_B[ch];
    auto load = [&](int quad) -> apt {
        const int row = (quad >> 1) * hb + r, col = (quad & 1) * hl + c;
        if (top) {
            apt inf;
            inf.x = fe_zero();
            inf.y = fe_zero();
            if (row >= n0 || col >= l0) return inf;
            return load_affine(par, ld_par, pt, (int64_t)row * l0 + col);
        }
        return load_aff_m(par, ld_par, pt, q * nb * lb + (int64_t)row * lb + col);
    };
    jpt R = jpt_from_affine(load(cb.qa));
    if (cb.sb != 0) {
        apt Q = load(cb.qb);
        if (cb.sb < 0) Q = apt_neg(Q);
        R = jpt_add_affine(R, Q);
    }
    store_jac_m(out, ld_out, pt, e_out, R);
}

// Leaves: leaf L computes its mb x lb block of products a (mb x nb, host
// plaintext sums) times its B block (nb x lb, internal affine), one lane per
// (leaf, i, j, point), ladder over the leaf's bit-width.
__global__ void __launch_bounds__(256) leaf_schoolbook_kernel(const int16_t *__restrict__ A, const int8_t *leaf_bits,
                                                              int64_t leaves, int mb, int nb, int lb,
                                                              const uint32_t *__restrict__ Bl, int64_t ld_b,
                                                              uint32_t *__restrict__ out, int64_t ld_out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per_leaf = (int64_t)mb * lb * 2;
    if (t >= leaves * per_leaf) return;
    const int64_t L = t / per_leaf;
    const int64_t rem = t - L * per_leaf;
    const int j = (int)(rem % lb);
    const int pt = (int)((rem / lb) & 1);
    const int i = (int)(rem / (2 * (int64_t)lb));
    const int bits = leaf_bits[L];
    const int16_t *a_row = A + (L * mb + i) * nb;
    jpt acc = jpt_infinity();
    for (int k = 0; k < nb; ++k) {
        const int a = a_row[k];
        if (a == 0) continue;
        apt b = load_aff_m(Bl, ld_b, pt, L * nb * lb + (int64_t)k * lb + j);
        if (a < 0) b = apt_neg(b);
        acc = jpt_add(acc, ladder_small((uint32_t)(a < 0 ? -a : a), bits, b));
    }
    store_jac_m(out, ld_out, pt, L * mb * lb + (int64_t)i * lb + j, acc);
}

// Level d + 1 -> d of the C side: the parent's quadrant Q of node q is the
// signed sum of its children's outputs.  Children (Jacobian, internal):
// nodes*7 blocks of hm x hl.  Parent: nodes blocks of (2 hm) x (2 hl),
// internal Jacobian; at the top the parent is the m0 x l0 result (cropped),
// Jacobian internal or canonical.
__global__ void __launch_bounds__(256) merge_c_kernel(const uint32_t *__restrict__ kids, int64_t ld_kids,
                                                      int64_t nodes, int hm, int hl, uint32_t *__restrict__ par,
                                                      int64_t ld_par, int top, int m0, int l0, int canonical) {
    const int64_t per_quad = (int64_t)hm * hl;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = nodes * 4 * per_quad * 2;
    if (t >= total) return;
    const int pt = (int)(t & 1);
    const int64_t e = t >> 1;
    const int64_t qq = e / per_quad;
    const int64_t rem = e - qq * per_quad;
    const int r = (int)(rem / hl), c = (int)(rem % hl);
    const int64_t q = qq / 4;
    const int quad = (int)(qq % 4);
    const quad_c qc = QUAD_C[quad];
    jpt acc = jpt_infinity();
    for (int x = 0; x < qc.n; ++x) {
        jpt M = load_jac_m(kids, ld_kids, pt, (q * 7 + qc.child[x]) * per_quad + rem);
        if (qc.sign[x] < 0) M = jpt_neg(M);
        acc = jpt_add(acc, M);
    }
    const int row = (quad >> 1) * hm + r, col = (quad & 1) * hl + c;
    if (top) {
        if (row >= m0 || col >= l0) return;
        const int64_t eo = (int64_t)row * l0 + col;
        if (canonical) store_jac(par, ld_par, pt, eo, acc);
        else store_jac_m(par, ld_par, pt, eo, acc);
    } else {
        store_jac_m(par, ld_par, pt, q * (int64_t)(2 * hm) * (2 * hl) + (int64_t)row * (2 * hl) + col, acc);
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
int64_t ld64(int64_t n) { return std::max<int64_t>(64, (n + 63) / 64 * 64); }

int64_t pow7(int d) {
    int64_t p = 1;
    while (d-- > 0) p *= 7;
    return p;
}

struct strassen_geom {
    int D = 0;
    int mp = 0, np = 0, lp = 0;  // padded shape
    // byte offsets in the workspace
    std::vector<size_t> off_b;   // B side, levels 1..D (internal affine), index d
    std::vector<int64_t> ld_b;
    size_t off_jtmp = 0;         // Jacobian child level before normalisation
    int64_t ld_jtmp = 0;
    size_t off_norm = 0, norm_bytes = 0;
    std::vector<size_t> off_c;   // C side, levels 0..D (internal Jacobian), index d (level 0 only for affine C)
    std::vector<int64_t> ld_c;
    size_t off_a = 0, a_bytes = 0, off_bits = 0;
    size_t total = 0;
};

int auto_depth(int m, int n, int l) {
    int D = 0;
    while (D < 6 && std::min({m, n, l}) / (1 << (D + 1)) >= 64) ++D;
    return D;
}

strassen_geom make_geom(int m, int n, int l, int D, int c_form) {
    strassen_geom G;
    G.D = D;
    const int s = 1 << D;
    G.mp = (m + s - 1) / s * s;
    G.np = (n + s - 1) / s * s;
    G.lp = (l + s - 1) / s * s;
    size_t off = 0;
    G.off_b.assign(D + 1, 0);
    G.ld_b.assign(D + 1, 0);
    int64_t jmax = 0, norm_max = 0;
    for (int d = 1; d <= D; ++d) {
        const int64_t elems = pow7(d) * (int64_t)(G.np >> d) * (G.lp >> d);
        G.ld_b[d] = ld64(elems);
        G.off_b[d] = off;
        off += align256((size_t)AFF2_PLANES * G.ld_b[d] * 4);
        jmax = std::max(jmax, G.ld_b[d]);
        norm_max = std::max<int64_t>(norm_max, elems);
    }
    G.ld_jtmp = jmax;
    G.off_jtmp = off;
    off += align256((size_t)JAC2_PLANES * jmax * 4);
    G.off_c.assign(D + 1, 0);
    G.ld_c.assign(D + 1, 0);
    for (int d = D; d >= 0; --d) {
        if (d == 0 && c_form != PCMM_AFFINE) break;  // Jacobian C is written directly
        const int64_t elems = d == 0 ? (int64_t)m * l : pow7(d) * (int64_t)(G.mp >> d) * (G.lp >> d);
        G.ld_c[d] = ld64(elems);
        G.off_c[d] = off;
        off += align256((size_t)JAC2_PLANES * G.ld_c[d] * 4);
        if (d == 0) norm_max = std::max<int64_t>(norm_max, elems);
    }
    G.norm_bytes = normalize_scratch_bytes(std::max<int64_t>(norm_max, 1), 2);
    G.off_norm = off;
    off += align256(G.norm_bytes);
    const int64_t leaves = pow7(D);
    G.a_bytes = (size_t)leaves * (G.mp >> D) * (G.np >> D) * 2;
    G.off_a = off;
    off += align256(G.a_bytes);
    G.off_bits = off;
    off += align256((size_t)leaves);
    G.total = off + 256;
    return G;
}

// The plaintext side of the recursion: the 7^D leaf matrices (exact integer
// sums), each mb x nb, in leaf order (child index fastest at the deepest
// level), and every leaf's bit-width (bits of its largest magnitude).
void expand_a(const std::vector<int32_t> &A0, int mp, int np, int D, std::vector<int16_t> &leaves,
              std::vector<int8_t> &bits, int *max_bits) {
    std::vector<std::vector<int32_t>> level{A0};
    int rows = mp, cols = np;
    for (int d = 0; d < D; ++d) {
        const int hr = rows / 2, hc = cols / 2;
        std::vector<std::vector<int32_t>> next;
        next.reserve(level.size() * 7);
        for (const auto &M : level) {
            auto quad = [&](int qd, int i, int k) { return M[(size_t)((qd >> 1) * hr + i) * cols + (qd & 1) * hc + k]; };
            // children in the order M1..M7: A11+A22, A21+A22, A11, A22, A11+A12, A21-A11, A12-A22
            const int qa[7] = {0, 2, 0, 3, 0, 2, 1};
            const int sb[7] = {+1, +1, 0, 0, +1, -1, -1};
            const int qb[7] = {3, 3, 0, 0, 1, 0, 3};
            for (int ch = 0; ch < 7; ++ch) {
                std::vector<int32_t> S((size_t)hr * hc);
                for (int i = 0; i < hr; ++i)
                    for (int k = 0; k < hc; ++k)
                        S[(size_t)i * hc + k] = quad(qa[ch], i, k) + (sb[ch] ? sb[ch] * quad(qb[ch], i, k) : 0);
                next.push_back(std::move(S));
            }
        }
        level = std::move(next);
        rows = hr;
        cols = hc;
    }
    const size_t per = (size_t)rows * cols;
    leaves.resize(level.size() * per);
    bits.resize(level.size());
    *max_bits = 1;
    for (size_t L = 0; L < level.size(); ++L) {
        int mx = 0;
        for (size_t x = 0; x < per; ++x) {
            leaves[L * per + x] = (int16_t)level[L][x];
            mx = std::max(mx, std::abs(level[L][x]));
        }
        int b = 1;
        while ((1 << b) <= mx) ++b;
        bits[L] = (int8_t)b;
        *max_bits = std::max(*max_bits, b);
    }
}

struct staging {
    void *host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
};
std::mutex g_lock;
staging g_stage[64];

bool valid_cfg(const pcmm_strassen_cfg *cfg) { return !cfg || (cfg->depth >= 0 && cfg->depth <= 6); }

int cfg_depth(const pcmm_strassen_cfg *cfg, int m, int n, int l) {
    if (cfg && cfg->depth > 0) return cfg->depth;
    return auto_depth(m, n, l);
}

}  // namespace

extern "C" pcmm_status pcmm_strassen_workspace(int32_t m, int32_t n, int32_t l, int32_t c_form,
                                               const pcmm_strassen_cfg *cfg, size_t *bytes) {
    if (!bytes || m < 0 || n < 0 || l < 0 || !valid_cfg(cfg) || (c_form != PCMM_AFFINE && c_form != PCMM_JACOBIAN))
        return PCMM_EINVAL;
    const int D = cfg_depth(cfg, m, n, l);
    *bytes = D == 0 ? pcmm_schoolbook_workspace(m, n, l, c_form) : make_geom(m, n, l, D, c_form).total;
    return PCMM_OK;
}

extern "C" pcmm_status pcmm_strassen(const void *A, int32_t m, int32_t n, int32_t bits, int32_t is_signed,
                                     const pcmm_mat *B, pcmm_mat *C, const pcmm_strassen_cfg *cfg,
                                     void *workspace, size_t ws_bytes, pcmm_strassen_stats *stats, void *stream) {
    if (!B || !C || m < 0 || n < 0 || bits < 1 || bits > 16 || !valid_cfg(cfg)) return PCMM_EINVAL;
    if (B->rows != n || B->cols < 0 || B->npts != 2 || B->form != PCMM_AFFINE) return PCMM_EINVAL;
    const int l = B->cols;
    const int64_t n_out = (int64_t)m * l;
    if (B->ld < (int64_t)n * l || ((int64_t)n * l > 0 && !B->d)) return PCMM_EINVAL;
    if (C->rows != m || C->cols != l || C->npts != 2 || (C->form != PCMM_AFFINE && C->form != PCMM_JACOBIAN))
        return PCMM_EINVAL;
    if (C->ld < n_out || (n_out > 0 && !C->d)) return PCMM_EINVAL;
    if (B->d == C->d && n_out > 0 && (int64_t)n * l > 0) return PCMM_EINVAL;
    if ((int64_t)m * n > 0 && !A) return PCMM_EINVAL;
    const int D = cfg_depth(cfg, m, n, l);
    if (stats) {
        memset(stats, 0, sizeof *stats);
        stats->depth = D;
        stats->leaf_bits = bits;
        stats->leaves = 1;
    }
    if (D == 0) return pcmm_schoolbook(A, m, n, bits, is_signed, B, C, workspace, ws_bytes, stream);
    const strassen_geom G = make_geom(m, n, l, D, C->form);
    // plaintext side: validate, pad, expand (host)
    const int lo = is_signed ? -(1 << (bits - 1)) : 0;
    const int hi = is_signed ? (1 << (bits - 1)) - 1 : (1 << bits) - 1;
    std::vector<int32_t> A0((size_t)G.mp * G.np, 0);
    for (int i = 0; i < m; ++i)
        for (int k = 0; k < n; ++k) {
            const int v = plain_at(A, (int64_t)i * n + k, bits, is_signed != 0);
            if (v < lo || v > hi) return PCMM_ERANGE;
            A0[(size_t)i * G.np + k] = v;
        }
    if (n_out == 0) return PCMM_OK;
    std::vector<int16_t> leafA;
    std::vector<int8_t> leafbits;
    int max_bits = 1;
    expand_a(A0, G.mp, G.np, D, leafA, leafbits, &max_bits);
    if (max_bits > 15) return PCMM_ERANGE;  // leaf sums must stay 16-bit signed
    if (stats) {
        stats->leaf_bits = max_bits;
        stats->leaves = pow7(D);
        // point operations executed: ciphertext block sums (5 per node and
        // level on the B side, 8 on the C side) and the leaf products
        int64_t adds = 0;
        for (int d = 0; d < D; ++d) {
            adds += pow7(d) * 5 * (int64_t)(G.np >> (d + 1)) * (G.lp >> (d + 1)) * 2;
            adds += pow7(d) * 8 * (int64_t)(G.mp >> (d + 1)) * (G.lp >> (d + 1)) * 2;
        }
        stats->block_adds = adds;
        int64_t ladder_ops = 0;
        const int64_t per = (int64_t)(G.mp >> D) * (G.np >> D);
        for (size_t L = 0; L < leafbits.size(); ++L) {
            int64_t nz = 0;
            for (int64_t x = 0; x < per; ++x) nz += leafA[L * per + x] != 0;
            ladder_ops += nz * (G.lp >> D) * 2 * 2 * leafbits[L];
        }
        stats->leaf_ladder_ops = ladder_ops;
    }
    if (!workspace || ws_bytes < G.total) return PCMM_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    int dev = 0;
    PCMM_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return PCMM_EDEVICE;
    {
        // leaf plaintexts and bit-widths through the device's pinned staging
        std::lock_guard<std::mutex> guard(g_lock);
        staging &sg = g_stage[dev];
        const size_t need = G.a_bytes + leafbits.size();
        if (sg.done) PCMM_HIP_TRY(hipEventSynchronize(sg.done));
        if (sg.bytes < need) {
            if (sg.host) (void)hipHostFree(sg.host);  // replaced by a larger buffer
            sg.host = nullptr;
            sg.bytes = 0;
            PCMM_HIP_TRY(hipHostMalloc(&sg.host, need, hipHostMallocDefault));
            sg.bytes = need;
        }
        if (!sg.done) PCMM_HIP_TRY(hipEventCreateWithFlags(&sg.done, hipEventDisableTiming));
        memcpy(sg.host, leafA.data(), G.a_bytes);
        memcpy((char *)sg.host + G.a_bytes, leafbits.data(), leafbits.size());
        PCMM_HIP_TRY(hipMemcpyAsync(ws + G.off_a, sg.host, G.a_bytes, hipMemcpyHostToDevice, s));
        PCMM_HIP_TRY(hipMemcpyAsync(ws + G.off_bits, (char *)sg.host + G.a_bytes, leafbits.size(),
                                    hipMemcpyHostToDevice, s));
        PCMM_HIP_TRY(hipEventRecord(sg.done, s));
    }
    // B side, level by level
    uint32_t *jtmp = (uint32_t *)(ws + G.off_jtmp);
    for (int d = 0; d < D; ++d) {
        const int64_t nodes = pow7(d);
        const int nb = G.np >> d, lb = G.lp >> d;
        const uint32_t *par = d == 0 ? B->d : (const uint32_t *)(ws + G.off_b[d]);
        const int64_t ld_par = d == 0 ? B->ld : G.ld_b[d];
        const int64_t child_elems = nodes * 7 * (int64_t)(nb / 2) * (lb / 2);
        const int64_t threads = child_elems * 2;
        if (threads > 0) {
            hipLaunchKernelGGL(split_b_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, par, ld_par,
                               d == 0 ? 1 : 0, n, l, nodes, nb, lb, jtmp, G.ld_jtmp);
            PCMM_LAUNCH_CHECK();
            pcmm_status st = launch_normalize(jtmp, G.ld_jtmp, true, (uint32_t *)(ws + G.off_b[d + 1]),
                                              G.ld_b[d + 1], true, child_elems, 2, ws + G.off_norm, G.norm_bytes, s);
            if (st != PCMM_OK) return st;
        }
    }
    // leaves
    const int64_t leaves = pow7(D);
    const int mb = G.mp >> D, nb = G.np >> D, lb = G.lp >> D;
    const bool affine = C->form == PCMM_AFFINE;
    uint32_t *leaf_out = (uint32_t *)(ws + G.off_c[D]);
    const int64_t ld_leaf = G.ld_c[D];
    {
        const int64_t threads = leaves * mb * lb * 2;
        const uint32_t *Bl = (const uint32_t *)(ws + G.off_b[D]);
        hipLaunchKernelGGL(leaf_schoolbook_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                           (const int16_t *)(ws + G.off_a), (const int8_t *)(ws + G.off_bits), leaves, mb, nb, lb,
                           Bl, G.ld_b[D], leaf_out, ld_leaf);
        PCMM_LAUNCH_CHECK();
    }
    // C side, level by level up to the top
    for (int d = D - 1; d >= 0; --d) {
        const int64_t nodes = pow7(d);
        const int hm = G.mp >> (d + 1), hl = G.lp >> (d + 1);
        const int64_t threads = nodes * 4 * (int64_t)hm * hl * 2;
        const bool top = d == 0;
        uint32_t *par = top ? (affine ? (uint32_t *)(ws + G.off_c[0]) : C->d) : (uint32_t *)(ws + G.off_c[d]);
        const int64_t ld_par = top ? (affine ? G.ld_c[0] : C->ld) : G.ld_c[d];
        hipLaunchKernelGGL(merge_c_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                           (const uint32_t *)(ws + G.off_c[d + 1]), G.ld_c[d + 1], nodes, hm, hl, par, ld_par,
                           top ? 1 : 0, m, l, (top && !affine) ? 1 : 0);
        PCMM_LAUNCH_CHECK();
    }
    if (affine)
        return launch_normalize((uint32_t *)(ws + G.off_c[0]), G.ld_c[0], true, C->d, C->ld, false, n_out, 2,
                                ws + G.off_norm, G.norm_bytes, s);
    return PCMM_OK;
}
