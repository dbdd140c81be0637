/* hlf.h -- C ABI of the MI355X (gfx950) FS2D HLF library, libhlf.so.
 *
 * The library solves the full-sampling 2D hidden linear function problem
 * (paper: "High-performance parallel classical scheme for simulating shallow
 * quantum circuits", Sections 1-2): given an n x n symmetric binary matrix A,
 * produce every z in {0,1}^n with q(x) = 2 z^T x (mod 4) for all x in Ker(A),
 * where q(x) = x^T A x mod 4 over the integers.  The solution set is the
 * affine space l XOR Col(A) with 2^r members, r = rank of A over GF(2)
 * (Section 2).
 *
 * Stage 1 (the paper's CLA module, Section 2 tasks (1)-(4)) is hlf_factor.
 * Stage 2 (the paper's classical parallel circuit, Section 2, Eqs. (1)-(3)) is
 * hlf_enumerate / hlf_enumerate_reduce, which traverse the 2^r inputs R^(r);
 * hlf_sample draws single uniform solutions, the output distribution of the
 * quantum circuit (Appendix A).
 *
 * ---------------------------------------------------------------------------
 * Conventions (shared by every entry point)
 * ---------------------------------------------------------------------------
 * Bit vectors.  A vector of n bits is W = ceil(n/64) little-endian uint64
 *   words; bit j (word j/64, bit j%64) is z_{j+1}, i.e. vertex j (0-based).
 *   Bits at positions >= n ("pad bits") are zero in every output and must be
 *   zero in every input.
 * Packed matrix.  rows[i*W + w] holds word w of row i of A: bit j of row i is
 *   A_ij.
 * Pivots P.  The ascending pivot columns of the reduced row echelon form of A
 *   over GF(2): the lexicographically first maximal independent column set
 *   (task (1)).  It does not depend on the elimination order.
 * Basis.  B_k = column p_k of A (= row p_k, A symmetric), k = 0..r-1.
 * Kernel basis.  For the free columns f (not in P), ascending: k_f has a 1 at
 *   f, 0 at every other free column and RREF[k][f] at pivot p_k (task (2)).
 * Shift l.  The unique solution with l_p = 0 for all p in P; l_f = q(k_f)/2
 *   for every free column f (tasks (3)-(4)).
 * Order.  Solution number i, 0 <= i < 2^r, is
 *       z_i = l XOR ( XOR_{k : bit k of g(i) is set} B_k ),  g(i) = i ^ (i>>1),
 *   the Gray-code traversal of R^(r) = (R_{p_1}..R_{p_r}); successive
 *   solutions differ by B_{ctz(i)}.
 * Hash.  h(z) = h_W with h_0 = 0, h_{w+1} = mix13(h_w ^ z_w ^ 0x9E3779B97F4A7C15),
 *   where mix13(x): x ^= x>>30; x *= 0xBF58476D1CE4E5B9; x ^= x>>27;
 *   x *= 0x94D049BB133111EB; x ^= x>>31 (all mod 2^64) -- the output function
 *   of SplitMix64 (Stafford's Mix13).  The hash of a set of solutions is the
 *   sum of h(z) mod 2^64, so it does not depend on the order and is additive
 *   over disjoint index ranges.
 * Sampling coefficients.  Word w (< R64 = ceil(r/64)) of the coefficient vector
 *   of sample s is the SplitMix64 output number s*R64 + w for the state that
 *   starts at `seed`: mix13(seed + (s*R64 + w + 1) * 0x9E3779B97F4A7C15); bits
 *   at positions >= r are cleared.  Sample s is l XOR (XOR_{bit k of c_s} B_k).
 *
 * Memory and streams.  Every pointer named *_dev is caller-owned device memory
 *   on the current HIP device; the library does not allocate, free or keep any
 *   of it.  The single-instance entry points never allocate; a batch (below)
 *   allocates its own result arrays once, in hlf_batch_create.  Every call is asynchronous on the caller's stream and returns once
 *   the work is enqueued.  Calls on different streams are independent; calls
 *   that write the same buffers must be ordered by the caller.
 *
 * Errors.  A host-detectable error (NULL pointer, n out of range, bad
 *   word_bits or flags) is returned at once and nothing is enqueued.
 *   Device-detectable errors are written to the factor record's status word:
 *   HLF_ENOTSYM for a matrix that is not symmetric or has nonzero pad bits,
 *   HLF_ERANGE for an index range outside [0, 2^r) or r > 62 in enumerate.
 *   Every later kernel that reads a record whose status is not HLF_OK does
 *   nothing (it writes no output), so a caller can enqueue a whole pipeline
 *   and check `status` once after synchronising.  A failed launch returns
 *   HLF_EDEVICE.
 */
#ifndef HLF_H
#define HLF_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hlf_status {
    HLF_OK = 0,
    HLF_EINVAL = -1,      /* bad argument (host-detected)                       */
    HLF_ENOTSYM = -2,     /* A not symmetric / not 0-1 / nonzero pad bits        */
    HLF_ERANGE = -3,      /* index range outside [0, 2^r), or r > 62            */
    HLF_ENOMEM = -4,      /* a capacity limit was exceeded                       */
    HLF_EDEVICE = -5,     /* a HIP call failed                                   */
    /* -6 is not used: no call can be cancelled once enqueued                    */
    HLF_EINTERNAL = -7    /* an internal invariant failed (q odd on Ker(A))      */
} hlf_status;

#define HLF_MAX_N 1024          /* largest n accepted by hlf_factor             */
#define HLF_MAX_WORDS 16        /* ceil(HLF_MAX_N / 64)                          */
#define HLF_MAX_ENUM_RANK 62    /* largest r for enumerate / reduce              */

/* Flags of hlf_enumerate_reduce. */
#define HLF_ACCUMULATE 1u       /* add into counts/hash/xorfold instead of overwriting */

/* Flags of hlf_factor_ex. */
#define HLF_FACTOR_WORKGROUP 1u   /* force the workgroup (LDS) variant for any n   */
#define HLF_FACTOR_PACK_STATUS 2u /* f->status holds the hlf_pack_dense verdict    */

/* Flags of hlf_enumerate_ex. */
#define HLF_ORDER_COUNTER 1u    /* binary-counter order (Section 4) instead of Gray */

/* Device-resident factor record (paper Section 2, tasks (1)-(4)).  The host
 * fills n and words and points the remaining members at caller-owned device
 * buffers of the stated sizes; hlf_factor writes them.                         */
typedef struct hlf_factors {
    int32_t n;          /* number of vertices, 1 .. HLF_MAX_N                      */
    int32_t words;      /* W = ceil(n / 64)                                        */
    int32_t *status;    /* dev [1]: hlf_status of the record                       */
    int32_t *rank;      /* dev [1]: r                                              */
    int32_t *pivots;    /* dev [n]: p_0 < ... < p_{r-1}; entries r..n-1 are -1     */
    uint64_t *basis;    /* dev [n*W]: rows 0..r-1 hold B_k; other rows untouched   */
    uint64_t *shift;    /* dev [W]: l                                              */
    uint64_t *kernel;   /* dev [n*W] or NULL: rows 0..n-r-1 hold k_f (f ascending) */
} hlf_factors;

/* Library version, (major << 16) | minor. */
int32_t hlf_version(void);

/* Human-readable name of a status code (static storage). */
const char *hlf_status_string(int32_t status);

/* ceil(n / 64): words per packed row or vector. */
int32_t hlf_words_for(int32_t n);

/* Pack and validate a dense matrix (the input of Section 1).
 *   A_dev      dev uint8 [n*n], row-major, entries 0 or 1.
 *   n          1 .. HLF_MAX_N.
 *   rows_dev   dev uint64 [n*W] output, packed rows (pad bits zero).
 *   status_dev dev int32 [1] output: HLF_OK, or HLF_ENOTSYM if A is not
 *              symmetric or holds a value other than 0 and 1.
 * Returns HLF_EINVAL for NULL pointers or n out of range.                       */
hlf_status hlf_pack_dense(const uint8_t *A_dev, int32_t n, uint64_t *rows_dev,
                          int32_t *status_dev, hipStream_t stream);

/* Stage 1, the CLA module (Section 2, tasks (1)-(4)): GF(2) Gauss-Jordan
 * elimination of the packed rows giving r and P, the Ker(A) basis, q(k_f) and
 * the canonical shift l, and the column-space basis B_k.
 *   rows_dev   dev uint64 [n*W], packed A (read only).
 *   f          host pointer to a record whose n, words and buffers are set;
 *              f->kernel may be NULL.  The record is read at call time only.
 * Writes f->status (HLF_OK, HLF_ENOTSYM, or HLF_EINTERNAL), f->rank,
 * f->pivots, f->basis, f->shift and, if not NULL, f->kernel.  Any n up to
 * HLF_MAX_N; n <= 192 runs one wavefront per instance, larger n one workgroup.
 * Returns HLF_EINVAL for NULL pointers, n out of range or words != ceil(n/64). */
hlf_status hlf_factor(const uint64_t *rows_dev, const hlf_factors *f, hipStream_t stream);

/* hlf_factor with flags.  HLF_FACTOR_WORKGROUP selects the workgroup variant
 * for every n (the results are identical).  HLF_FACTOR_PACK_STATUS: the caller
 * passed f->status as the status_dev of an hlf_pack_dense of these rows
 * enqueued earlier on the same stream; if that verdict is not HLF_OK it stays
 * in f->status and nothing else of the record is written (the packed rows of
 * an invalid matrix are not factored), else the call behaves as without the
 * flag.  This saves merging the two verdicts after the call.                   */
hlf_status hlf_factor_ex(const uint64_t *rows_dev, const hlf_factors *f, uint32_t flags,
                         hipStream_t stream);

/* Stages 1 and 2 of one small instance in one launch (Sections 1-2: the
 * validation of A, tasks (1)-(4) and the traversal of Eq. (3)): the result of
 * hlf_pack_dense + hlf_factor + hlf_enumerate, for n <= 64.
 *   A_dev      dev uint8 [n*n], row-major, entries 0 or 1 (as hlf_pack_dense).
 *   f          record with n <= 64 (words = 1); written as by hlf_factor.
 *   begin, count, word_bits, out_dev  as hlf_enumerate with a uint16/uint32/
 *              uint64 word per solution (word_bits 16, 32 or 64, >= n), begin
 *              a multiple of 16 / (word_bits / 8) and out_dev 16-byte aligned.
 * Device errors: HLF_ENOTSYM (invalid A) or HLF_ERANGE (r > 62 or begin +
 * count > 2^r) in f->status, and nothing is written to out_dev.  count = 0
 * runs stage 1 only.  Every workgroup of the launch factors the instance
 * itself, so no workgroup waits for another: meant for latency-bound small
 * counts (for large counts hlf_factor + hlf_enumerate factor once).
 * Returns HLF_EINVAL for NULL pointers, n > 64, a word size not allowed for n,
 * or a misaligned begin or out_dev.                                            */
hlf_status hlf_solve_dense(const uint8_t *A_dev, const hlf_factors *f, uint64_t begin,
                           uint64_t count, int32_t word_bits, void *out_dev, hipStream_t stream);

/* Stage 2, materialise (Section 2, the traversal of R^(r) through Eq. (3) and
 * the final CNOT layer): out[i - begin] = z_i for i in [begin, begin + count).
 *   word_bits  16, 32 or 64 when n <= word_bits <= 64: one uint16/uint32/uint64
 *              per solution; or 64*W for any n: W uint64 words per solution.
 *   out_dev    dev buffer of count * word_bits / 8 bytes; the fast path needs
 *              16-byte alignment (any alignment is correct).
 * Device errors: HLF_ERANGE in f->status if r > 62 or begin + count > 2^r
 * (nothing is written).  count = 0 enqueues nothing and returns HLF_OK.
 * Returns HLF_EINVAL for NULL pointers or word_bits not allowed for n.          */
hlf_status hlf_enumerate(const hlf_factors *f, uint64_t begin, uint64_t count,
                         int32_t word_bits, void *out_dev, hipStream_t stream);

/* hlf_enumerate with flags.  HLF_ORDER_COUNTER: solution number i is
 * z_i = l XOR (XOR over set bits k of i of B_k), the output of the paper's
 * circuit fed by the binary counter of the FPGA design (Section 4); the
 * circuit is defined for the graph of any symmetric A (Section 5), and this
 * is its output for every A (the tile algebra runs on the prefix sums
 * B_0 ^ ... ^ B_k, whose Gray-order walk is the counter order of B).
 * Without flags: hlf_enumerate (Gray order).  Arguments, errors as there.
 * Returns HLF_EINVAL for unknown flags.                                         */
hlf_status hlf_enumerate_ex(const hlf_factors *f, uint64_t begin, uint64_t count,
                            int32_t word_bits, uint32_t flags, void *out_dev,
                            hipStream_t stream);

/* Stage 2 as the paper's circuit, evaluated literally (Section 2, Eqs. (1)-(2),
 * Fig. 1(c)) in the binary-counter order of the FPGA design (Section 4):
 * for i in [begin, begin + count), R carries bit k of i at the pivot position
 * p_k and 0 elsewhere; y_v = XOR of R_u over the grid neighbours u of v, XOR
 * b_v R_v (the four edge layers and the Toffoli layer); out[i - begin] =
 * y XOR l (the final CNOT layer).  Equivalently z = l XOR (XOR over set bits
 * k of i of B_k): the same solution set as hlf_enumerate in another order.
 *   rows_dev  packed A (as for hlf_factor); A must be a subgraph of the
 *             grid_N x grid_N grid, n = grid_N^2 <= HLF_MAX_N, vertices
 *             row-major (else HLF_EINVAL in f->status, nothing written).
 *   word_bits n <= 64: 16/32/64 with n <= word_bits, begin a multiple of
 *             16/(word_bits/8) and a 16-byte aligned out_dev; n > 64: 64*W
 *             (W uint64 words per solution, 8-byte aligned out_dev).  Else
 *             HLF_EINVAL.
 * Device errors as hlf_enumerate.                                               */
hlf_status hlf_enumerate_circuit(const hlf_factors *f, const uint64_t *rows_dev, int32_t grid_N,
                                 uint64_t begin, uint64_t count, int32_t word_bits, void *out_dev,
                                 hipStream_t stream);

/* Stage 2, reduce: over the solutions z_i, i in [begin, begin + count),
 *   counts_dev  dev uint64 [n]: counts[j] = number of solutions with bit j set;
 *   hash_dev    dev uint64 [1]: sum of h(z_i) mod 2^64;
 *   xorfold_dev dev uint64 [W] or NULL: XOR of all z_i.
 * Outputs are overwritten, or added to (counts, hash: mod 2^64; xorfold: XOR)
 * with HLF_ACCUMULATE, so disjoint ranges can be reduced one after another.
 * Device errors as hlf_enumerate.  count = 0 with overwrite zeroes the outputs. */
hlf_status hlf_enumerate_reduce(const hlf_factors *f, uint64_t begin, uint64_t count,
                                uint32_t flags, uint64_t *counts_dev, uint64_t *hash_dev,
                                uint64_t *xorfold_dev, hipStream_t stream);

/* Uniform single solutions, as the quantum circuit outputs them (Section 1,
 * Appendix A): out[s*W .. s*W+W-1] = l XOR (XOR_{bit k of c_s} B_k),
 * s = 0 .. num-1.
 *   seed       state of the SplitMix64 coefficient stream (see Conventions).
 *   coeffs_dev NULL, or dev uint64 [num * ceil(r/64)]: explicit coefficient
 *              vectors (bits >= r ignored), r being the rank in the record.
 *   out_dev    dev uint64 [num * W].
 * Works for any r (no 62-bit limit).  num = 0 enqueues nothing.                 */
hlf_status hlf_sample(const hlf_factors *f, uint64_t seed, uint64_t num,
                      const uint64_t *coeffs_dev, uint64_t *out_dev, hipStream_t stream);

/* Verification data (Section 5: the ideal output distribution as the input
 * of a cross-entropy benchmark of a device running the circuit).
 *
 * Pair statistics of a uniform solution z, exact for any r:
 *   quarters_dev[i*n + j] = 4 * P(z_i = 1 and z_j = 1) (uint8, n*n entries);
 * the diagonal holds 4 * P(z_i = 1).  Closed form: with A_i the rows of A,
 * 0 if A_i = 0 or A_j = 0 (then z_i = 0 or z_j = 0 always), 2 if A_i = A_j
 * is nonzero (then z_i = z_j always), else 1 (independent uniform bits).
 *   rows_dev  the packed rows the record f was factored from (n x W words).
 * Gated on f->status: nothing is written unless it is HLF_OK.
 * Returns HLF_EINVAL for NULL pointers or a malformed record.                   */
hlf_status hlf_pair_stats(const hlf_factors *f, const uint64_t *rows_dev, uint8_t *quarters_dev,
                          hipStream_t stream);

/* Membership: member_dev[s] = 1 if z_s = z_dev[s*W .. s*W+W-1] is a solution
 * (the problem's definition, Section 1: q(x) = 2 z.x mod 4 for every x in
 * Ker(A); on the kernel basis k_f this is <k_f, z> = l_f mod 2), else 0.
 * The ideal probability of z_s is 2^-r * member_dev[s], and the linear
 * cross-entropy estimate over S samples is 2^(n-r) * (sum of member) / S - 1.
 *   f         record with a kernel buffer (f->kernel != NULL), filled by
 *             hlf_factor.  num = 0 enqueues nothing.
 * Gated on f->status: nothing is written unless it is HLF_OK.
 * Returns HLF_EINVAL for NULL pointers, f->kernel == NULL or a malformed record. */
hlf_status hlf_membership(const hlf_factors *f, const uint64_t *z_dev, uint64_t num,
                          uint8_t *member_dev, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batches: many instances of mixed n handled by one launch per stage (the
 * FS2D workload over a set of grid instances, Sections 1-2 applied per
 * instance).  A batch owns its device result arrays; they are allocated once
 * by hlf_batch_create (not on the hot path) and freed by hlf_batch_destroy.
 *
 * Input layout: the dense matrices of all instances concatenated, instance i
 * as a row-major n_i x n_i uint8 block at byte offset dense_off[i] = sum of
 * n_k^2 over k < i.  Result layout (offsets reported by hlf_batch_get_layout):
 * instance i's record fields sit at mat_off[i] (basis, kernel: n_i*W_i
 * words), vec_off[i] (shift: W_i words) and piv_off[i] (pivots, counts: n_i
 * entries); status, rank and hash are indexed by i.
 * ------------------------------------------------------------------------- */
typedef struct hlf_batch_s *hlf_batch;

typedef struct hlf_batch_layout {
    int32_t count;             /* number of instances I                          */
    int32_t max_n;             /* largest n_i                                    */
    int64_t dense_bytes;       /* sum n_i^2: bytes of the concatenated input     */
    int64_t mat_words;         /* sum n_i * W_i                                  */
    int64_t vec_words;         /* sum W_i                                        */
    int64_t piv_entries;       /* sum n_i                                        */
    const int64_t *dense_off;  /* host [I], owned by the batch                   */
    const int64_t *mat_off;    /* host [I]                                       */
    const int64_t *vec_off;    /* host [I]                                       */
    const int64_t *piv_off;    /* host [I]                                       */
    int32_t *status;           /* dev [I]                                        */
    int32_t *rank;             /* dev [I]                                        */
    int32_t *pivots;           /* dev [piv_entries]                              */
    uint64_t *basis;           /* dev [mat_words]                                */
    uint64_t *shift;           /* dev [vec_words]                                */
    uint64_t *kernel;          /* dev [mat_words]                                */
    uint64_t *counts;          /* dev [piv_entries]: reduce counts               */
    uint64_t *hash;            /* dev [I]: reduce hash                           */
} hlf_batch_layout;

/* Launch parameters of hlf_batch_reduce: chunks of 2^chunk_log2 solutions
 * (10..30) are the unit of dynamic scheduling; waves_per_cu (1..16) sizes the
 * persistent grid.  hlf_batch_tune picks both by timing the real batch.       */
typedef struct hlf_batch_params {
    int32_t chunk_log2;
    int32_t waves_per_cu;
} hlf_batch_params;

/* Create a batch of `count` (1..2^20) instances with n_host[i] vertices
 * (1..HLF_MAX_N) on the current device.  Allocates the device arrays.
 * Returns HLF_EINVAL for bad arguments, HLF_ENOMEM if allocation fails.       */
hlf_status hlf_batch_create(int32_t count, const int32_t *n_host, hlf_batch *out);

/* Free a batch (waits for the device).  NULL is accepted.                     */
hlf_status hlf_batch_destroy(hlf_batch b);

/* Offsets and device pointers of a batch.                                     */
hlf_status hlf_batch_get_layout(hlf_batch b, hlf_batch_layout *layout);

/* Stage 1 for every instance (pack + validate + factor, Section 1 and
 * Section 2 tasks (1)-(4)): one launch for all instances with n_i <= 192 (a
 * wavefront each), one workgroup launch per larger instance.  A_dev is the
 * concatenated dense input.  Writes every record field of every instance.     */
hlf_status hlf_batch_factor_dense(hlf_batch b, const uint8_t *A_dev, hipStream_t stream);

/* Stage 2 materialise for `num` instances at once: out[k][i - begin[k]] = z_i
 * of instance inst[k] for i in [begin[k], begin[k] + count[k]).  inst, begin,
 * count and out are host arrays of length num; out[k] are device buffers.
 * word_bits 16/32/64 with n_i <= word_bits for every listed instance.  Device
 * errors go to the instance's status as in hlf_enumerate.                    */
hlf_status hlf_batch_enumerate(hlf_batch b, int32_t num, const int32_t *inst,
                               const uint64_t *begin, const uint64_t *count, void *const *out,
                               int32_t word_bits, hipStream_t stream);

/* hlf_batch_enumerate for batch b, plus stage 1 (as hlf_batch_factor_dense)
 * of every instance of another batch `next` (all n <= 64) from its dense
 * input A_next_dev, carried by the same launch: extra workgroups factor
 * `next` while the others materialise b.  Nothing in the launch reads the
 * records it writes, so a pipeline alternates two batches: launch k
 * materialises the instances factored by launch k-1 and factors those of
 * launch k+1.  With S streams taking the steps in turn, launch k factors for
 * launch k+S on the same stream, 2S batches in rotation and a separate output
 * set per stream: no launch then touches the records or outputs of the
 * launches running beside it, and each one's start-up and drain overlap the
 * others'.  next must differ from b (HLF_EINVAL otherwise).                  */
hlf_status hlf_batch_enumerate_overlap(hlf_batch b, int32_t num, const int32_t *inst,
                                       const uint64_t *begin, const uint64_t *count,
                                       void *const *out, int32_t word_bits, hlf_batch next,
                                       const uint8_t *A_next_dev, hipStream_t stream);

/* Stage 1 and stage 2 materialise in ONE launch, for instances with
 * n_i <= word_bits <= 64: every listed instance is packed, validated and
 * factored (its record written as by hlf_batch_factor_dense) and then
 * out[k][i - begin[k]] = z_i for i in [begin[k], begin[k] + count[k]).
 * The first workgroup of an instance factors it while the instance's other
 * workgroups wait for that result.  1 <= num <= 16 tasks, each with count > 0,
 * begin a multiple of 16 / (word_bits/8) and a 16-byte aligned out[k]
 * (HLF_EINVAL otherwise).  Calls on one batch must be ordered (one stream).   */
hlf_status hlf_batch_solve(hlf_batch b, const uint8_t *A_dev, int32_t num, const int32_t *inst,
                           const uint64_t *begin, const uint64_t *count, void *const *out,
                           int32_t word_bits, hipStream_t stream);

/* Stage 1 + stage 2 reduce for the whole batch in ONE persistent launch (plus
 * one small launch that resets its work queue): wavefronts first take factor
 * tasks; every instance with rank <= max_rank (<= 62) then publishes its
 * 2^r solutions as chunks on a device queue, which all wavefronts drain.
 * Results: counts[piv_off[i] + j], hash[i] over all 2^r_i solutions (zero
 * for instances with r_i > max_rank).  Needs max_n <= 192 (else HLF_EINVAL).
 * params NULL selects defaults (or the tuned values, if hlf_batch_tune ran).
 * The queue counts chunks in 40 bits: HLF_EINVAL unless
 * count * 2^max(0, max_rank - chunk_log2) < 2^40 (count = instances).         */
hlf_status hlf_batch_reduce(hlf_batch b, const uint8_t *A_dev, int32_t max_rank,
                            const hlf_batch_params *params, hipStream_t stream);

/* Autotuner: times hlf_batch_reduce on this batch over a grid of
 * (chunk_log2, waves_per_cu) candidates on `stream` (synchronising it) and
 * stores the fastest as the batch default; *best and *best_ms receive it.
 * Every candidate produces the same results.  Candidates whose chunk count
 * would not fit the queue (see hlf_batch_reduce) are skipped; HLF_EINVAL if
 * none fits.                                                                  */
hlf_status hlf_batch_tune(hlf_batch b, const uint8_t *A_dev, int32_t max_rank,
                          hlf_batch_params *best, float *best_ms, hipStream_t stream);

/* Capture hlf_batch_reduce(b, A_dev, max_rank, params) into a HIP graph owned
 * by the batch (replacing a previous one) and replay it with
 * hlf_batch_graph_launch.  A_dev must stay valid while the graph is used.    */
hlf_status hlf_batch_graph_capture(hlf_batch b, const uint8_t *A_dev, int32_t max_rank,
                                   const hlf_batch_params *params);
hlf_status hlf_batch_graph_launch(hlf_batch b, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Serving: continuous admission of single-instance requests (Section 1's
 * problem per request: stage 1, then every solution when 2^r is small --
 * the traversal of Section 2 -- or uniform samples, the output distribution
 * of Appendix A).  A server owns a worker thread, `slots` HIP streams, one
 * device arena of hbm_bytes (every device byte the server uses: inputs,
 * packed rows, stage-1 records, outputs and the stage-1 cache) and one pinned
 * host arena of host_bytes for results.  A request is admitted when its
 * arrival time has passed, a slot is free and its stage-1 memory (input,
 * packed rows, record) can be carved from the arena; its phases then run on
 * the slot's stream, and once r is known its output is carved at its exact
 * size (the request waits while the arena or the result arena is full).  A
 * request's result depends only on (A, seed).
 * ------------------------------------------------------------------------- */
typedef struct hlf_server_s *hlf_server;

typedef struct hlf_server_config {
    int32_t slots;          /* concurrent requests (HIP streams), 1 .. 64           */
    int64_t hbm_bytes;      /* device arena, >= 1 MiB                               */
    int64_t host_bytes;     /* pinned result arena, >= 1 MiB                        */
    int32_t num_samples;    /* samples per sampling request, >= 1                   */
    int32_t enum_max_rank;  /* all solutions when n <= 64 and r <= this (0 .. 30)    */
    int32_t cache_entries;  /* stage-1 records kept (LRU), 0 = no cache              */
} hlf_server_config;

typedef struct hlf_request {
    int64_t id;             /* caller's tag, returned in the result                 */
    int32_t n;              /* 1 .. HLF_MAX_N                                       */
    const uint8_t *A;       /* host [n*n] row-major 0/1, read at admission: it must
                               stay valid until the request's result is polled   */
    uint64_t seed;          /* sampling seed (hlf_sample's stream)                  */
    uint64_t key[2];        /* stage-1 cache key (a digest of A); {0,0}: no caching */
    int64_t arrival_ns;     /* not admitted before this time of hlf_server_now      */
} hlf_request;

typedef struct hlf_result {
    int64_t id;
    int32_t status;         /* hlf_status: HLF_OK, HLF_ENOTSYM, HLF_ENOMEM, ...      */
    int32_t n, rank;
    int32_t kind;           /* 1: all solutions, 2: samples, 0: error (no data)      */
    int32_t word_bytes;     /* bytes per solution: 2/4/8 (kind 1), 8*W (kind 2)      */
    int64_t count;          /* solutions in data                                    */
    const void *data;       /* pinned host memory of the server, valid until
                               hlf_server_release(data)                             */
    int64_t arrival_ns, admitted_ns, finished_ns;  /* server clock                  */
    int32_t cache_hit;
} hlf_result;

typedef struct hlf_server_stats {
    int64_t admitted, completed, cache_hits;
    int64_t hbm_bytes;       /* the arena                                           */
    int64_t hbm_peak_bytes;  /* most arena bytes in use at once                     */
    int64_t host_peak_bytes; /* most pinned result bytes in use at once             */
    int32_t worker_status;   /* HLF_OK, or the first HIP failure of the worker      */
} hlf_server_stats;

/* Create a server on the current device (allocates its arenas and streams and
 * starts its worker).  HLF_EINVAL for a bad configuration, HLF_ENOMEM if an
 * arena cannot be allocated.                                                  */
hlf_status hlf_server_create(const hlf_server_config *cfg, hlf_server *out);

/* Nanoseconds since the server was created (its clock for arrival times).     */
int64_t hlf_server_now(hlf_server s);

/* Queue `count` requests (the request records are copied; each A is read
 * when its request is admitted).  Requests are admitted in submission order.  HLF_EINVAL for n outside
 * [1, HLF_MAX_N] or a NULL A (nothing is queued then).  A request whose
 * worst-case memory exceeds the arena completes with HLF_ENOMEM.              */
hlf_status hlf_server_submit(hlf_server s, const hlf_request *reqs, int32_t count);

/* Move up to `max` finished results to out (completion order), waiting up to
 * wait_ms for the first; *got receives the number moved.                      */
hlf_status hlf_server_poll(hlf_server s, hlf_result *out, int32_t max, int32_t *got,
                           int32_t wait_ms);

/* Return a result's pinned memory to the server.  Results that are never
 * released fill the host arena, and requests then wait for memory.           */
hlf_status hlf_server_release(hlf_server s, const void *data);

hlf_status hlf_server_get_stats(hlf_server s, hlf_server_stats *out);

/* Stop admitting, finish the requests in flight, free everything (the pinned
 * result memory included).  NULL is accepted.                                 */
hlf_status hlf_server_destroy(hlf_server s);

/* hlf_batch_reduce without a batch object, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * the allocator): the call allocates nothing and frees nothing.  Its scratch
 * (work queue, chunk slots, layout offsets: about 832 KiB) is a device array
 * of the library, one per GPU, kept until the process ends.  Every call on a
 * GPU uses that GPU's array: calls that overlap on one GPU (on different
 * streams) race and must be ordered by the caller.
 *   count      instances, 1 .. 16384 (HLF_EINVAL beyond).
 *   max_n      an upper bound of every n_i, 1 .. 192 (HLF_EINVAL otherwise).
 *   n_dev      dev int32 [count]: n_i.  An entry outside [1, max_n] takes no
 *              space in the layout and gets status HLF_EINVAL.
 *   A_dev      dev uint8: the dense matrices concatenated, instance i at
 *              byte offset sum_{k<i} n_k^2 (the layout of hlf_batch).
 *   outputs    caller-owned device arrays in the layout of
 *              hlf_batch_get_layout for these n_i: status_dev, rank_dev,
 *              hash_dev [count]; pivots_dev, counts_dev [sum n_i];
 *              basis_dev [sum n_i W_i]; shift_dev [sum W_i]; kernel_dev
 *              [sum n_i W_i] or NULL.
 *   params     NULL (chunk_log2 20, 8 waves per CU) or explicit.
 * Results as hlf_batch_reduce; the same limits on max_rank and the chunk
 * count apply (HLF_EINVAL).                                                    */
hlf_status hlf_batch_reduce_noalloc(int32_t count, int32_t max_n, const int32_t *n_dev,
                                    const uint8_t *A_dev, int32_t max_rank,
                                    const hlf_batch_params *params, int32_t *status_dev,
                                    int32_t *rank_dev, int32_t *pivots_dev, uint64_t *basis_dev,
                                    uint64_t *shift_dev, uint64_t *kernel_dev,
                                    uint64_t *counts_dev, uint64_t *hash_dev, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HLF_H */
