/*
 * pcmm.h -- plaintext-ciphertext matrix multiplication (PC-MM) over unpacked
 * EC-ElGamal ciphertexts on NIST P-256, on AMD Instinct MI355X (gfx950).
 *
 * The problem (Alg. 3 of the paper, Sec. 3.3): given a plaintext m x n integer
 * matrix A and n l EC-ElGamal ciphertexts Enc(b_kj) = (B1_kj, B2_kj), produce
 * the m l ciphertexts Enc(c_ij) with c_ij = sum_k a_ik b_kj, i.e. in the group
 * of points
 *     (C1_ij, C2_ij) = (sum_k a_ik B1_kj, sum_k a_ik B2_kj).
 * Two methods are provided: the schoolbook inner products with every product
 * a_ik B_kj computed by the Montgomery ladder (Sec. 3.1, Alg. 1) and Cussen's
 * compression-reconstruction (Alg. 2 inside Alg. 3).  Both give identical
 * group elements; after pcmm_normalize the bytes are identical too.
 *
 * Scheme (Sec. 2.4): KeyGen picks x in [1, q-1] and H = xG; Encrypt(m) =
 * (rG, rH + mG) with r in [1, q-1]; decryption recovers mG = C2 - x C1 (the
 * bounded discrete logarithm that turns mG into m is not part of this API).
 *
 * ------------------------------------------------------------------------
 * Conventions
 *   Errors      every call returns a pcmm_status; 0 is success.  Arguments are
 *               validated on the host before any work is queued; invalid
 *               arguments queue nothing.  GPU work is asynchronous on the given
 *               stream (a hipStream_t passed as void*; NULL = the null stream);
 *               launch failures return PCMM_EDEVICE.
 *   Ownership   the caller allocates and frees every buffer (device matrices,
 *               workspaces, host arrays).  The library keeps only immutable
 *               curve tables per device, created on first use.
 *   Aliasing    inputs and outputs must not overlap unless a call says so.
 *   Points      device points are structure-of-arrays 32-bit little-endian
 *               limbs in canonical form (integers in [0, p), not Montgomery):
 *                 affine   : 2 coordinates (x, y); infinity = (0, 0)
 *                 jacobian : 3 coordinates (X, Y, Z); x = X/Z^2, y = Y/Z^3;
 *                            infinity <=> Z = 0
 *               Element e of a pcmm_mat with `npts` points per element stores
 *               limb `w` of coordinate `c` of point `pt` at
 *                 d[((pt * form + c) * 8 + w) * ld + e]
 *               so each limb plane is contiguous over elements (coalesced).
 *   Ints        plaintext matrices A are host arrays, row-major, whose element
 *               width follows the declared bit-width t = `bits` (1..16):
 *               int8 (signed) / uint8 (unsigned) for t <= 8, int16 / uint16
 *               for 9 <= t <= 16.  Entries must satisfy 0 <= a < 2^t
 *               (unsigned) or -2^(t-1) <= a < 2^(t-1) (signed), else
 *               PCMM_ERANGE.  Cussen column groups of g > 3 need t <= 8.
 *               Keeping n max|a| max|b| below the message bound of the
 *               decryptor (Sec. 2.4) is the caller's duty.
 * ------------------------------------------------------------------------
 */
#ifndef PCMM_H
#define PCMM_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PCMM_OK = 0,
    PCMM_EINVAL = -1,       /* bad shape, bit-width, form, null pointer, config */
    PCMM_ERANGE = -2,       /* an entry of A outside its declared bit-width     */
    PCMM_ENOMEM = -3,       /* caller workspace too small                      */
    PCMM_EDEVICE = -4,      /* HIP runtime or launch error                     */
    PCMM_ENOTONCURVE = -5,  /* a host point is not on P-256                    */
    PCMM_ETOOLARGE = -6     /* needs more than the library's static scratch    */
} pcmm_status;

#define PCMM_AFFINE 2
#define PCMM_JACOBIAN 3

/* Host form of a point: big-endian affine coordinates; infinity = (0, 0). */
typedef struct {
    uint8_t x[32];
    uint8_t y[32];
} pcmm_point_be;

/* A device matrix of points (see Conventions). */
typedef struct {
    int32_t rows, cols;  /* logical shape; element e = r * cols + c              */
    int32_t npts;        /* points per element: 2 for ciphertexts, 1 for points  */
    int32_t form;        /* PCMM_AFFINE or PCMM_JACOBIAN (coordinates per point) */
    int64_t ld;          /* limb-plane stride in elements, >= rows * cols        */
    uint32_t *d;         /* device memory, caller-owned                          */
} pcmm_mat;

/* Tuning of pcmm_cussen.  Zero fields take the library's choice.
 *   rounds  N, compression rounds of Alg. 2 (default 4, as in the paper; 1..8)
 *   group   columns of A per code (default 1 = Alg. 3 exactly, one column of A
 *           per compression; g > 1 compresses row segments of g columns into
 *           one code and builds the table of their ciphertext combinations;
 *           1..4, or PCMM_GROUP_AUTO: the autotuner builds the plans for
 *           g = 1..4 and keeps the one of least predicted GPU time, from a
 *           cost model of the persistent accumulation (row chains and tile
 *           rounds), the digit combinations (throughput, or a lane's chain
 *           when lanes are few) and the split-k reduction, fitted to MI355X
 *           kernel times; the choice of g and k_split is cached per
 *           (m, n, l, bits, signedness, rounds, requested k_split) for the
 *           process, and a cached g > 1 whose tables exceed the autotuner's
 *           size cap on another matrix of that shape falls back to g = 1;
 *           entries of 9..16 bits allow g <= 3)
 *   k_split split of the n (inner) dimension over independent partial sums that
 *           are then added (a power of two <= 64; 0 = the split of least
 *           predicted time under the same cost model)
 *   k_chunk column groups per code list of the accumulation; each list is
 *           padded to its longest row (0 = one list per split of n)
 *   profile nonzero: record HIP events around every launch of the call on
 *           its stream, wait for them, and return per-stage durations in the
 *           stats (the call then returns after its GPU work has finished)
 *   stage_events  NULL, or an array of PCMM_STAGE_EVENTS hipEvent_t handles
 *           owned by the caller (created with timing enabled).  The call
 *           records the boundaries of its stages into them on its stream --
 *           before the plan upload, after it, after the table build, the
 *           accumulation, the split-k reduction and the normalisation -- and
 *           does not wait for them, so consecutive calls still overlap host
 *           planning with GPU work.  The caller reads the durations with
 *           hipEventElapsedTime once the stream has reached the last one.
 *           With profile nonzero as well, these events are the ones waited
 *           on and read into the stats. */
#define PCMM_STAGE_EVENTS 6
#define PCMM_GROUP_AUTO (-1)
typedef struct {
    int32_t rounds;
    int32_t group;
    int32_t k_split;
    int32_t k_chunk;
    int32_t profile;
    void **stage_events;
} pcmm_cussen_cfg;

/* Operation counts of one pcmm_cussen call, derived from its plan. */
typedef struct {
    int64_t level_mults;     /* sum over columns of n_N (ECSMs per ciphertext point)       */
    int64_t level_adds;      /* sum over columns of sum_{w<N} n_w (paper's counting)        */
    int64_t table_entries;   /* sum over groups of table entries per output column (digit
                                tables and, for g > 1, digit combinations)               */
    int64_t table_adds;      /* point additions executed per output column to build tables
                                (digit-table prefix sums and combinations)               */
    int64_t accum_adds;      /* mixed additions executed per output column (all rows)      */
    int64_t max_entries;     /* largest table (entries) of one column (group)              */
    int64_t workspace_bytes; /* device workspace of this problem's tables, scratch and
                                partial sums within a plan run (0 without GPU work)      */
    int64_t combo_adds;      /* of table_adds: combinations of digits (g > 1), each one
                                affine addition of two table entries                     */
    int64_t digit_entries;   /* of table_entries: entries of the columns' digit tables    */
    int32_t k_split;         /* split of the inner dimension that was used                 */
    int32_t lanes_per_chain; /* table-build batch: output columns (chains) per lane        */
    int32_t group;           /* columns of A per code that was used (after autotuning)     */
    int32_t coop_lanes;      /* lanes sharing each level-1 prefix-sum chain of the table
                                build in this run (0: one lane per chain, up to 64); a
                                run of single-column groups with few output columns
                                splits each chain into blocks, each lane starting its
                                block at its first entry's multiple of the base point   */
    /* with cfg->profile: milliseconds from the first to the last event of each stage */
    float ms_upload, ms_table, ms_accumulate, ms_reduce, ms_normalize, ms_total;
} pcmm_cussen_stats;

/* KeyGen (Sec. 2.4): x = scalar(seed, domain 0, index 0) in [1, q-1] and the
 * public point H = xG.  Scalars come from a counter-based derivation: with
 * SplitMix64's output function mix(), base = mix(seed ^ (domain << 56) ^ idx),
 * w_i = mix(base + (i + 1) * 0x9E3779B97F4A7C15) for i = 0..4,
 * X = sum_i w_i 2^(64 i), scalar = X mod (q - 1) + 1.
 * sk_be: 32 bytes big-endian (host).  pk: host.  Runs on the current device
 * and returns after the result is on the host. */
pcmm_status pcmm_keygen(uint64_t seed, uint8_t sk_be[32], pcmm_point_be *pk);

/* Encrypt (Sec. 2.4): element e (row-major index of the rows x cols message
 * matrix) gets r_e = scalar(seed, domain 1, idx0 + e) and
 * ct_e = (r_e G, r_e H + m_e G), with m_e taken mod q (negative allowed).
 * msg_dev: device int32, rows x cols row-major.  ct_out: rows x cols, npts 2,
 * PCMM_AFFINE.  workspace: device scratch of pcmm_encrypt_workspace() bytes
 * (holds the fixed-base table of H).  PCMM_ENOTONCURVE if pk is not a
 * finite point of P-256. */
pcmm_status pcmm_encrypt(const pcmm_point_be *pk, const int32_t *msg_dev, int32_t rows,
                         int32_t cols, uint64_t seed, int64_t idx0, pcmm_mat *ct_out,
                         void *workspace, size_t ws_bytes, void *stream);
size_t pcmm_encrypt_workspace(void);

/* Schoolbook PC-MM (Sec. 3.1): C_ij = sum_k a_ik B_kj, each term by the
 * Montgomery ladder of Alg. 1 over the t bits of |a_ik| (negative a_ik act on
 * -B_kj), accumulated by point additions.  A: host m x n.  B: device n x l
 * ciphertexts, affine.  C: device m x l ciphertexts, PCMM_JACOBIAN (write-only;
 * run pcmm_normalize for canonical affine bytes) or PCMM_AFFINE (normalised
 * here through `workspace`).  workspace: pcmm_schoolbook_workspace() bytes. */
pcmm_status pcmm_schoolbook(const void *A, int32_t m, int32_t n, int32_t bits,
                            int32_t is_signed, const pcmm_mat *B, pcmm_mat *C,
                            void *workspace, size_t ws_bytes, void *stream);
size_t pcmm_schoolbook_workspace(int32_t m, int32_t n, int32_t l, int32_t c_form);

/* Cussen PC-MM (Alg. 3 with Alg. 2): per column (group) of A, compress the
 * magnitudes by N rounds of sort / de-duplicate / difference, build the table
 * of ciphertext multiples T_kj[u] = u B_kj by the reconstruction's prefix
 * sums, then C_ij += sign(a_ik) T_kj[code_ik].  Same arguments as
 * pcmm_schoolbook plus cfg (NULL = defaults) and a workspace of
 * pcmm_cussen_workspace() bytes (plan, tables, partial sums).  stats may be
 * NULL; when given it receives the plan's operation counts.  The plan is
 * built on host threads and copied through a ring of 4 pinned buffers per
 * device: the call may block until the copy of the call 4 before it (not its
 * kernels) has executed, so consecutive calls overlap their host work with
 * the GPU and the host may run up to 4 calls ahead. */
pcmm_status pcmm_cussen(const void *A, int32_t m, int32_t n, int32_t bits, int32_t is_signed,
                        const pcmm_mat *B, pcmm_mat *C, const pcmm_cussen_cfg *cfg,
                        void *workspace, size_t ws_bytes, pcmm_cussen_stats *stats,
                        void *stream);
pcmm_status pcmm_cussen_workspace(const void *A, int32_t m, int32_t n, int32_t l, int32_t bits,
                                  int32_t is_signed, int32_t c_form, const pcmm_cussen_cfg *cfg,
                                  size_t *bytes);

/* pcmm_cussen for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, hosts that forbid hipMalloc): the same
 * kernels and results as pcmm_cussen, with the workspace taken from a static
 * device array of PCMM_STATIC_SCRATCH_BYTES that the library holds on every
 * GPU it runs on until the process ends.  The call allocates no device or
 * pinned memory and creates no HIP objects; the caller still owns B and C.
 *   - A problem whose pcmm_cussen_workspace() exceeds
 *     PCMM_STATIC_SCRATCH_BYTES returns PCMM_ETOOLARGE before any device call.
 *   - cfg->profile must be 0 (PCMM_EINVAL otherwise); caller-owned
 *     cfg->stage_events are recorded as in pcmm_cussen.
 *   - The plan image is copied from pageable host memory, so the call returns
 *     once that copy has been made (it waits for the stream's earlier work);
 *     the kernels run asynchronously.
 *   - Every call on one GPU uses that GPU's single array, which keeps the last
 *     call's contents (each call initialises what it reads).  Calls on one
 *     stream are ordered; calls that overlap on one GPU (other streams, other
 *     threads) race on the array and give undefined results. */
#define PCMM_STATIC_SCRATCH_BYTES (64u << 20)
pcmm_status pcmm_cussen_static(const void *A, int32_t m, int32_t n, int32_t bits, int32_t is_signed,
                               const pcmm_mat *B, pcmm_mat *C, const pcmm_cussen_cfg *cfg,
                               pcmm_cussen_stats *stats, void *stream);

/* Compiled plans: one or more Cussen PC-MMs, compressed once on the host and
 * run any number of times (a static plaintext A served against fresh
 * ciphertexts), or many uneven PC-MMs run together.  A run queues the same
 * few kernels whatever the number of problems: one table build over all
 * problems, one persistent accumulation kernel whose workgroups take
 * (problem, row tile, pair tile, split) tiles from a device queue, one
 * split-k reduction and one affine normalisation.  When the problems' tables
 * and partial sums together exceed 14 GB, the problems are packed into
 * phases of at most that size (first fit, largest first; a larger problem
 * is a phase of its own) that run those kernels one after another on one
 * shared workspace region, so the workspace is the largest phase's, not the
 * sum.  The plan's host image
 * (plans and per-problem geometry) is immutable after creation and is copied
 * to the workspace at the start of every run, so a run can be captured into
 * a hipGraph and replayed (the matrices and workspace are those given at
 * capture).  A plan is bound to the device that was current at creation. */
#define PCMM_PLAN_MAX_PROBLEMS 64
typedef struct pcmm_plan_s *pcmm_plan;

typedef struct {
    const void *A;       /* host, m x n row-major (see PC-MM plaintexts), read only during pcmm_plan_create */
    int32_t m, n, l;     /* C = A B with B n x l                                     */
    int32_t bits, is_signed;
    int32_t c_form;      /* PCMM_AFFINE (canonical, normalised) or PCMM_JACOBIAN     */
    pcmm_cussen_cfg cfg; /* rounds, group (or PCMM_GROUP_AUTO), k_split, k_chunk; its
                            profile and stage_events fields are ignored here          */
} pcmm_problem;

/* Compresses every A (host threads over problems) and lays out the
 * workspace.  count: 1..PCMM_PLAN_MAX_PROBLEMS.  *out receives a handle that
 * pcmm_plan_destroy releases.  PCMM_ERANGE if an A entry is outside its
 * bit-width; PCMM_EINVAL for bad shapes or cfg; PCMM_ENOMEM if host memory
 * runs out. */
pcmm_status pcmm_plan_create(const pcmm_problem *problems, int32_t count, pcmm_plan *out);
pcmm_status pcmm_plan_destroy(pcmm_plan plan);
/* Device workspace bytes a run needs (tables, partial sums, the plan image). */
pcmm_status pcmm_plan_workspace(pcmm_plan plan, size_t *bytes);
/* Operation counts and the chosen geometry of problem `index`. */
pcmm_status pcmm_plan_stats(pcmm_plan plan, int32_t index, pcmm_cussen_stats *stats);
/* Runs every problem of the plan: B[i] (n_i x l_i affine ciphertexts) and
 * C[i] (m_i x l_i, the problem's c_form) are host arrays of `count` matrix
 * descriptors of device memory; B[i] and C[i] must not alias.  stage_events:
 * NULL or PCMM_STAGE_EVENTS caller-owned events recorded at the stage
 * boundaries (as in pcmm_cussen_cfg; with several phases the events after
 * the upload bracket the last phase's stages, and the earlier phases fall
 * in the table stage).  Queues the work on `stream` and
 * returns without waiting.  Runs that overlap on one workspace race. */
pcmm_status pcmm_plan_run(pcmm_plan plan, const pcmm_mat *B, pcmm_mat *C, void *workspace,
                          size_t ws_bytes, void **stage_events, void *stream);

/* Resident plans and selected runs (serving static layers).
 * pcmm_plan_make_resident copies the plan's compiled arrays once, on
 * `stream`, into caller-owned device memory of pcmm_plan_resident_bytes()
 * bytes, which must stay allocated and unchanged while the plan runs
 * selections; runs queued on other streams must be ordered after that copy.
 * pcmm_plan_run_selected then runs the problems which[0..k) of the plan
 * (1 <= k <= PCMM_PLAN_MAX_PROBLEMS; an index may repeat: every entry is an
 * independent PC-MM with its own B[r] and C[r]) with the same kernels as
 * pcmm_plan_run, uploading only a small block of descriptors per run.  The
 * workspace holds the selected problems' tables and partial sums
 * (pcmm_plan_selected_workspace(); the sum of their stats' workspace_bytes
 * plus a few KB).  Runs on different streams with different workspaces may
 * overlap on the device; up to 8 runs of one plan can be in flight before a
 * further call waits for the oldest to have started executing. */
pcmm_status pcmm_plan_resident_bytes(pcmm_plan plan, size_t *bytes);
pcmm_status pcmm_plan_make_resident(pcmm_plan plan, void *device_mem, size_t bytes, void *stream);
pcmm_status pcmm_plan_selected_workspace(pcmm_plan plan, const int32_t *which, int32_t k, size_t *bytes);
pcmm_status pcmm_plan_run_selected(pcmm_plan plan, const int32_t *which, int32_t k, const pcmm_mat *B,
                                   pcmm_mat *C, void *workspace, size_t ws_bytes, void **stage_events,
                                   void *stream);

/* Strassen PC-MM (Sec. 3.1): the 2 x 2 block recursion with seven block
 * products M1..M7 and C11 = M1 + M4 - M5 + M7, C12 = M3 + M5, C21 = M2 + M4,
 * C22 = M1 - M2 + M3 + M6, run breadth first to `depth` levels; the leaf
 * products use the schoolbook method (Alg. 1 per term, ladders over each
 * leaf's bit-width, which grows by at most one bit per level as the
 * plaintext blocks are summed).  The plaintext sums are formed on the host;
 * every ciphertext block sum and every leaf product runs on the GPU.  Shapes
 * that are not multiples of 2^depth are padded (zero plaintexts, infinity
 * ciphertexts) and C is cropped.  Same arguments as pcmm_schoolbook plus
 * cfg (NULL = defaults) and stats (may be NULL).  PCMM_ERANGE also when a
 * leaf plaintext would not fit 16-bit signed.
 *   depth  0 = automatic (as many levels as keep leaves >= 64 in every
 *          dimension; none for small shapes, which then run the schoolbook
 *          product), 1..6 = that many levels. */
typedef struct {
    int32_t depth;
    int32_t reserved;
} pcmm_strassen_cfg;

typedef struct {
    int32_t depth;            /* levels used                                  */
    int32_t leaf_bits;        /* largest bit-width of a leaf plaintext          */
    int64_t leaves;           /* 7^depth leaf products                        */
    int64_t block_adds;       /* point additions of the ciphertext block sums */
    int64_t leaf_ladder_ops;  /* ladder steps (addition + doubling) of the leaves */
} pcmm_strassen_stats;

pcmm_status pcmm_strassen(const void *A, int32_t m, int32_t n, int32_t bits, int32_t is_signed,
                          const pcmm_mat *B, pcmm_mat *C, const pcmm_strassen_cfg *cfg,
                          void *workspace, size_t ws_bytes, pcmm_strassen_stats *stats, void *stream);
pcmm_status pcmm_strassen_workspace(int32_t m, int32_t n, int32_t l, int32_t c_form,
                                    const pcmm_strassen_cfg *cfg, size_t *bytes);

/* Full decryption (Sec. 2.4): m = phi^-1(C2 - x C1) for phi(m) = m G, with
 * the message bound the scheme needs (|m| <= bound), by baby-step
 * giant-step.  The baby-step table holds j G for 0 <= j < 2^log2_baby
 * (4..24) and a hash index on x; it is built once on the GPU into
 * caller-owned device memory of pcmm_dlog_table_bytes() bytes
 * (pcmm_dlog_table_build, scratch of pcmm_dlog_table_workspace() bytes) and
 * serves every later decryption.  pcmm_decrypt writes, for each element e of
 * the affine ciphertext matrix C, the integer m_e to out[e] (device int64,
 * rows * cols, row-major), or INT64_MIN when |m_e| > bound (no match).  A
 * decryption costs one variable-base scalar multiplication per element plus
 * 2 ceil(bound / (2^(log2_baby + 1) - 1)) + 1 giant steps; bound must keep
 * the giant multiples below 2^32 * (2^(log2_baby + 1) - 1).  workspace:
 * pcmm_decrypt_workspace() bytes. */
pcmm_status pcmm_dlog_table_bytes(int32_t log2_baby, size_t *bytes);
pcmm_status pcmm_dlog_table_workspace(int32_t log2_baby, size_t *bytes);
pcmm_status pcmm_dlog_table_build(int32_t log2_baby, void *table, size_t bytes, void *workspace,
                                  size_t ws_bytes, void *stream);
pcmm_status pcmm_decrypt_workspace(int64_t elements, int64_t bound, int32_t log2_baby, size_t *bytes);
pcmm_status pcmm_decrypt(const uint8_t sk_be[32], const pcmm_mat *C, int64_t bound, const void *table,
                         size_t table_bytes, int32_t log2_baby, int64_t *out, void *workspace,
                         size_t ws_bytes, void *stream);

/* Host-only: the compression plan's operation counts for A (no GPU work).
 * With cfg->group = PCMM_GROUP_AUTO the autotuner assumes a square problem
 * (l = m output columns) for its choice. */
pcmm_status pcmm_cussen_plan_stats(const void *A, int32_t m, int32_t n, int32_t bits,
                                   int32_t is_signed, const pcmm_cussen_cfg *cfg,
                                   pcmm_cussen_stats *stats);

/* Normalise Jacobian points to canonical affine (x, y) = (X/Z^2, Y/Z^3) with
 * one field inversion per batch of points (Montgomery's simultaneous
 * inversion); infinity (Z = 0) becomes (0, 0).  in: PCMM_JACOBIAN; out:
 * PCMM_AFFINE, same rows, cols, npts.  out may alias in (same d and ld).
 * workspace: pcmm_normalize_workspace(rows * cols, npts) bytes. */
pcmm_status pcmm_normalize(const pcmm_mat *in, pcmm_mat *out, void *workspace, size_t ws_bytes,
                           void *stream);
size_t pcmm_normalize_workspace(int64_t elements, int32_t npts);

/* Decryption to points (Sec. 2.4): M_e = C2_e - x C1_e (= m_e G for a valid
 * ciphertext of m_e).  sk_be: 32 bytes big-endian, 1 <= x < q.  C: affine
 * ciphertexts (npts 2).  M: affine, npts 1, same rows and cols. */
pcmm_status pcmm_decrypt_to_points(const uint8_t sk_be[32], const pcmm_mat *C, pcmm_mat *M,
                                   void *stream);

const char *pcmm_strerror(pcmm_status s);

#ifdef __cplusplus
}
#endif
#endif
