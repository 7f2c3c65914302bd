/*
 * ssbh.h - sampled sub-block hashing on AMD Instinct MI355X (gfx950).
 *
 * The method (arXiv 2308.02856): a large weakly random bit block A^N is
 * divided into N_S sub-blocks by seeded random sampling (Sec. III.B step 1),
 * an over-long sub-block aborts the protocol (Sec. III.B step 2, Sec. III.D),
 * every sub-block is hashed with a GF(2) Toeplitz matrix (Sec. I, K = T.A';
 * Sec. III.B step 3) and the outputs are concatenated (Sec. III.B step 4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Bit strings: arrays of uint64_t words; bit k is (w[k >> 6] >> (k & 63)) & 1
 *   (least significant bit first).  Sub-block j of a sampled buffer starts at
 *   word d_word_off[j] and holds d_len[j] bits; bits past d_len[j] in its last
 *   word are zero after ssbh_sample and ignored by ssbh_hash_batch.
 * Toeplitz matrices (the paper fixes no placement of the seed bits; this
 *   library's convention):  T_j[r][c] = s[j*S + c - r + M - 1]  for
 *   0 <= r < m_j, 0 <= c < n_j, where s is the seed bit string, S the seed
 *   stride and M the row cap (M >= every m_j).  S = 0 means one shared seed:
 *   every T_j is the top-left m_j x n_j corner of one M x max(n_j) matrix.
 *   S >= max(n_j) + M - 1 gives every sub-block its own independent seed, as
 *   the paper's security claim requires (Sec. III.B step 3).  With one block
 *   and M = m this is T[r][c] = s[c - r + m - 1]: row r is the seed window
 *   that starts at bit m - 1 - r.
 * Indices are 0-based: the paper's V_i in [1, N_S] is V_i - 1 here.
 * Pointers named d_* are device memory owned by the caller; the library never
 *   frees them.  The library owns its scratch memory, sized on demand and
 *   released by ssbh_destroy.  Every call is asynchronous on the given HIP
 *   stream (a hipStream_t passed as void *, NULL = the null stream) unless
 *   stated otherwise.  Calls that share one context must not overlap: they
 *   share its scratch memory.
 * Errors: entry points return ssbh_status and never throw.  Argument errors
 *   that the host can see are returned at once, with a message in
 *   ssbh_last_error() and nothing enqueued.  Conditions that only the device
 *   can see (lengths, the abort rule) are written to a caller-owned device
 *   int32 d_status; every kernel of ssbh_hash_batch does nothing when
 *   *d_status is nonzero on entry, so an aborted sampling leaves d_out
 *   untouched.
 */
#ifndef SSBH_H
#define SSBH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ssbh_ctx ssbh_ctx;

typedef enum {
    SSBH_OK = 0,
    SSBH_PENDING = 1,              /* serving: job not finished yet          */
    SSBH_E_INVAL = -1,             /* bad argument or inconsistent lengths   */
    SSBH_E_ABORT_OVERSIZE = -2,    /* some n_j > L_S^UB (Sec. III.B step 2)  */
    SSBH_E_NOMEM = -3,             /* device memory or HBM budget exhausted  */
    SSBH_E_DEVICE = -4,            /* a HIP runtime call failed              */
    SSBH_E_UNKNOWN_JOB = -5,       /* serving: no such job id                */
    SSBH_E_UNSUPPORTED = -6,       /* outside this build's limits            */
    SSBH_E_PRECISION = -7          /* FFT hash: an output entry was not within
                                      1/4 of an integer (never expected; the
                                      output is then not trusted)            */
} ssbh_status;

/* Sampling modes (Sec. III.B step 1). */
enum {
    SSBH_SAMPLE_IID = 0,      /* V_i drawn on the device from SplitMix64     */
    SSBH_SAMPLE_PERMUTE = 1,  /* d_assign = permutation pi; contiguous split */
    SSBH_SAMPLE_EXPLICIT = 2  /* d_assign = V_i given by the caller          */
};

/* Output-length rules (Sec. III.B step 3). */
enum {
    SSBH_OUT_FIXED = 0,       /* m_j = out_a (the paper's l~)                 */
    SSBH_OUT_RATIO = 1,       /* m_j = floor(n_j * out_a / out_b)             */
    SSBH_OUT_EXPLICIT = 2     /* m_j = d_out_len[j]                           */
};

/* Hash kernels. */
enum {
    SSBH_K_AUTO = 0,          /* library picks (autotuned)                    */
    SSBH_K_VALU = 1,          /* bit-sliced AND-XOR + popcount parity         */
    SSBH_K_MFMA_I8 = 2,       /* int8 matrix cores, int32 sums, then mod 2;
                                 only for a shared seed (seed_stride == 0)    */
    SSBH_K_FFT = 3,           /* middle product by double-precision FFTs,
                                 every entry rounded and checked.  Shared
                                 seed of at most 2^31 bits: two sub-blocks
                                 per transform, four (x_lo + 2^18 x_hi per
                                 part) when seed_bits + 1 - m_cap < 2^18 and
                                 the transform length is at most 2^20
                                 (ssbh_set_fft_packing).  Seed stride S > 0 (at most
                                 2^31): one transform per sub-block carrying
                                 its own seed window (real) and its bits
                                 (imaginary), squared pointwise; needs every
                                 n_j + m_cap - 1 <= the transform length of
                                 S (true when S >= n_max + m_cap - 1), else
                                 *d_status = SSBH_E_UNSUPPORTED.  A single
                                 sub-block with a shared seed takes the same
                                 one-transform form (no seed spectrum)
                                 unless packing is forced.  Such transforms
                                 up to 2^18 points keep the data between
                                 passes as complex floats (arithmetic in
                                 double; error bound below the 1/4 checked,
                                 see ssbh_set_fft_storage)                  */
    SSBH_K_MFMA_F4 = 4        /* fp4 (e2m1) matrix cores, 64 columns per
                                 matrix op, fp32 sums (exact: the host
                                 requires seed_bits + 1 - m_cap <= 2^24, so
                                 every n_j <= 2^24), then mod 2; shared seed
                                 only; schedules with an even MT            */
};

/* Limits of this build. */
#define SSBH_MAX_SUB_LDS 16384u   /* n_sub limit of the i.i.d./explicit modes */
#define SSBH_MAX_SAMPLE_BITS 4293918720ull  /* 2^32 - 2^20: n_bits limit of one
                                               sampling call (32-bit indices) */

/* ------------------------------------------------------------- context --- */

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
 * device memory that the serving scheduler may hold for admitted jobs
 * (0 = 80% of the free memory at creation).  Returns SSBH_E_DEVICE when the
 * device cannot be used. */
ssbh_status ssbh_create(int device, uint64_t hbm_budget_bytes, ssbh_ctx **out);

/* Wait for the context's own work, stop its serving thread and free its
 * scratch memory and pending jobs.  NULL is ignored. */
void ssbh_destroy(ssbh_ctx *ctx);

/* Message of the last error on the calling thread ("" if none).  Valid until
 * the next call on the same thread. */
const char *ssbh_last_error(void);

/* Number of compute units of the context's device. */
int ssbh_num_cus(const ssbh_ctx *ctx);

/* --------------------------------------------------- sampling (a1 - a3) --- */

/* Divide n_bits input bits into n_sub sub-blocks (Sec. III.B step 1) and
 * apply the abort rule (Sec. III.B step 2, Sec. III.D).
 *
 *  d_in          input bits A^N (ceil(n_bits/64) words; bits past n_bits are
 *                ignored).
 *  mode          SSBH_SAMPLE_IID: V_i is drawn on the device from the
 *                SplitMix64 stream with key sample_key (output t is
 *                mix(key + (t+1)*0x9E3779B97F4A7C15) with Stafford's variant
 *                13 finaliser); round i uses the low 32 bits of output i/2
 *                for even i and the high 32 bits for odd i, and
 *                V_i = floor(u_i * n_sub / 2^32) (exactly uniform when n_sub
 *                is a power of two, relative bias below n_sub / 2^32
 *                otherwise).  Sub-block j holds the bits with V_i = j in
 *                ascending i.  n_sub <= SSBH_MAX_SUB_LDS.
 *                SSBH_SAMPLE_EXPLICIT: the same, with V_i = d_assign[i]
 *                (uint32, every value < n_sub, else *d_status = SSBH_E_INVAL).
 *                SSBH_SAMPLE_PERMUTE: B[k] = A[pi[k]] and sub-block j is
 *                B[jL, (j+1)L) with L = n_bits / n_sub (n_sub must divide
 *                n_bits).  pi is d_assign (a permutation of 0..n_bits-1,
 *                uint32; entries >= n_bits give *d_status = SSBH_E_INVAL)
 *                or, when d_assign is NULL, the keyed permutation of
 *                sample_key built on the device as ssbh_permutation does
 *                (scratch of about 16 bytes per input bit, held by the
 *                context, which keeps the permutation of the last
 *                (sample_key, n_bits) and builds it again only for another
 *                pair).  From 2^26 input bits the gather streams in
 *                three passes through about 14 bytes of context scratch per
 *                input bit (cells of window offsets, a slot per output bit,
 *                looked-up bits); when that cannot be reserved, or when the
 *                permutation overfills a cell (far outside a random
 *                permutation's spread), each output bit is read directly.
 *                The result is the same either way.  For the keyed
 *                permutation the first of the three passes (which depends
 *                on pi and n_sub only) is kept for the last
 *                (sample_key, n_bits, n_sub) and skipped when they repeat;
 *                a caller's d_assign is never cached.
 *  l_ub          L_S^UB; 0 disables the abort rule.  If some n_j > l_ub,
 *                *d_status = SSBH_E_ABORT_OVERSIZE.
 *  d_sub         output sub-blocks, sub_capacity_words words.  Needs
 *                ceil(n_bits/64) + n_sub words (IID, EXPLICIT) or
 *                n_sub * ceil(L/64) words (PERMUTE).
 *  d_len         output n_j (n_sub uint64).
 *  d_word_off    output W_j = sum_{k<j} ceil(n_k/64) (n_sub uint64).
 *  d_status      device int32, overwritten with 0 or an error code.
 *  stream        hipStream_t.
 * n_bits = 0 gives n_sub empty sub-blocks; n_bits above SSBH_MAX_SAMPLE_BITS
 * returns SSBH_E_UNSUPPORTED. */
ssbh_status ssbh_sample(ssbh_ctx *ctx, const uint64_t *d_in, uint64_t n_bits,
                        uint32_t n_sub, uint32_t mode, uint64_t sample_key,
                        const uint32_t *d_assign, uint64_t l_ub,
                        uint64_t *d_sub, uint64_t sub_capacity_words,
                        uint64_t *d_len, uint64_t *d_word_off,
                        int32_t *d_status, void *stream);

/* The keyed permutation of the permutation-split sampling mode (not in the
 * paper, which draws V_i i.i.d.; used by workloads that cut a permuted block
 * into equal sub-blocks): Durstenfeld's Fisher-Yates shuffle (CACM 7(7),
 * 1964, Algorithm 235) of the identity 0..n-1, which for k = n-1 down to 1
 * exchanges entries k and j_k, with j_k = floor(r_t * (k+1) / 2^64) and r_t
 * output t = n-1-k of the SplitMix64 stream of `key` (the stream defined
 * under ssbh_sample; multiply-shift without rejection, bias below
 * (k+1)/2^64).  The result is computed by parallel passes, not by the
 * sequential loop, and equals the loop's for every key.
 *  d_perm   output, n uint32 (device, caller-owned).
 *  n        at most SSBH_MAX_SAMPLE_BITS (else SSBH_E_UNSUPPORTED); 0 writes
 *           nothing.
 * Scratch: 12 bytes per entry, held by the context until ssbh_destroy. */
ssbh_status ssbh_permutation(ssbh_ctx *ctx, uint64_t key, uint64_t n,
                             uint32_t *d_perm, void *stream);

/* Sampling followed by sifting inside every sub-block (Sec. III.B steps 1-2)
 * and the abort rule.  d_keep holds one flag per round (n_bits bits, same
 * layout as d_in); sub-block j is the list of bits A_i with V_i = j and
 * keep_i = 1, in ascending i, which is what sifting each sampled sub-block
 * gives, since V_i is drawn for every round whether kept or not.  n_j and the
 * abort rule count kept bits only.  Modes SSBH_SAMPLE_IID and
 * SSBH_SAMPLE_EXPLICIT (SSBH_SAMPLE_PERMUTE gives SSBH_E_INVAL); every other
 * argument, the capacity rule and the error behaviour are those of
 * ssbh_sample. */
ssbh_status ssbh_sample_sifted(ssbh_ctx *ctx, const uint64_t *d_in,
                               const uint64_t *d_keep, uint64_t n_bits,
                               uint32_t n_sub, uint32_t mode,
                               uint64_t sample_key, const uint32_t *d_assign,
                               uint64_t l_ub, uint64_t *d_sub,
                               uint64_t sub_capacity_words, uint64_t *d_len,
                               uint64_t *d_word_off, int32_t *d_status,
                               void *stream);

/* Key length of a GEAT-analysed protocol (host only): the generalised
 * entropy accumulation bound (App. A) with the BBM92 min-tradeoff function
 * of App. C, tangent to the entropy bound at e_tangent, for direct hashing
 * (n_sub = 1) or for sampled sub-block hashing by Claim 1 (Sec. III.C): each
 * of n_sub sub-protocols has f / n_sub and l / n_sub, eps_sec = n_sub eps' +
 * eps_abort, and error-correction leakage and smoothing are split the same
 * way.  The result is the total key length in bits (n_sub times the
 * sub-protocol's), negative when no key can be extracted. */
typedef struct {
    double n_rounds;    /* N, rounds of the protocol                         */
    double p_x;         /* testing probability p_X (p_Z = 1 - p_X)           */
    double q_tol;       /* tolerated phase error rate                        */
    double eta_tol;     /* tolerated detection probability                   */
    double e_bit;       /* bit error rate (error-correction leakage)         */
    double f_ec;        /* error-correction efficiency (>= 1)                */
    double eps_sec;     /* secrecy of the whole protocol                     */
    double eps_sm;      /* smoothing parameter of the whole protocol         */
    double p_omega;     /* probability that the protocol passes              */
    double d_x;         /* dimension of the output register X_i              */
    double eps_abort;   /* abort chance eps_Omega' (sub-block method, else 0) */
    uint32_t n_sub;     /* N_S; 1 = direct hashing                           */
} ssbh_geat_params;

/* Key length at a fixed Renyi parameter alpha in (1, 1.5) and tangent point
 * e_tangent in (0, 0.5).  SSBH_E_INVAL for parameters outside their ranges
 * (see the field comments; also 2 eps_sm < eps_sec - eps_abort). */
ssbh_status ssbh_geat_key_length(const ssbh_geat_params *p, double alpha,
                                 double e_tangent, double *key_bits);

/* The largest key length over alpha and e_tangent (grid in log10(alpha - 1)
 * and log10(e_tangent), then golden-section refinement); alpha and
 * e_tangent (may be NULL) receive the maximiser. */
ssbh_status ssbh_geat_optimise(const ssbh_geat_params *p, double *key_bits,
                               double *alpha, double *e_tangent);

/* Abort threshold L_S^UB (Sec. III.D), computed on the host.  A sifted
 * sub-block's length is Binomial(n_rounds, p_sift) (p_sift = chance that a
 * round is kept AND lands in that sub-block); the binomial tail bound of
 * Sec. III.D gives P(length > L) <= 1 - Phi(sqrt(2 n H(L/n, p))) for
 * L >= n p, with H(x, p) = x ln(x/p) + (1-x) ln((1-x)/(1-p)).  A union bound
 * over the n_sub sub-blocks (the reading taken for the formula's undefined
 * m) gives eps(L) = n_sub * (1 - Phi(...)).
 *  *l_ub    receives the smallest integer L >= ceil(n p) with eps(L) <= eps
 *           (n_rounds if none is smaller: no sub-block can be longer);
 *  *eps_at  (may be NULL) receives eps(*l_ub).
 * Errors: SSBH_E_INVAL for p_sift outside (0, 1), eps <= 0, n_sub = 0,
 * n_rounds = 0 or a null l_ub. */
ssbh_status ssbh_ub_threshold(uint64_t n_rounds, double p_sift, uint32_t n_sub,
                              double eps, uint64_t *l_ub, double *eps_at);

/* ------------------------------------------- hash + concatenate (a4 - a7) --- */

/* Hash every sub-block with its Toeplitz matrix T_j and concatenate the
 * outputs (Sec. I; Sec. III.B steps 3-4):
 *     K_j[r] = XOR_{c < n_j} ( s[j*S + c - r + M - 1] AND x_j[c] ),
 *     K = K_0 || K_1 || ... ,  K_j at bit offset O_j = sum_{k<j} m_k.
 * n_sub = 1 is the plain single-block hash.
 *
 *  d_sub, d_len, d_word_off  sub-blocks as written by ssbh_sample (or built
 *                by the caller in the same layout); every sub-block must lie
 *                inside the first sub_capacity_words words of d_sub.
 *  out_rule, out_a, out_b, d_out_len   output lengths m_j (see SSBH_OUT_*;
 *                d_out_len is read only for SSBH_OUT_EXPLICIT).
 *  d_seed, seed_bits   seed bit string s.  Every sub-block with n_j > 0 and
 *                m_j > 0 needs j*S + n_j + M - 1 <= seed_bits.
 *  seed_stride   S (0 = shared seed).
 *  m_cap         M; every m_j must be <= M.
 *  kernel        SSBH_K_*.
 *  d_out         output, out_capacity_bits bits (ceil(/64) words); zeroed and
 *                then written; bits past the total are zero.
 *  d_out_total_bits  device uint64, receives sum_j m_j.
 *  d_status      device int32 (in/out): nonzero on entry makes the call a
 *                no-op on the device; a length, seed or capacity violation
 *                found on the device sets SSBH_E_INVAL and leaves d_out
 *                untouched.
 * The result is bit-identical for every kernel and schedule. */
ssbh_status ssbh_hash_batch(ssbh_ctx *ctx, const uint64_t *d_sub,
                            uint64_t sub_capacity_words,
                            const uint64_t *d_len, const uint64_t *d_word_off,
                            uint32_t n_sub, uint32_t out_rule, uint64_t out_a,
                            uint64_t out_b, const uint64_t *d_out_len,
                            const uint64_t *d_seed, uint64_t seed_bits,
                            uint64_t seed_stride, uint64_t m_cap,
                            uint32_t kernel, uint64_t *d_out,
                            uint64_t out_capacity_bits,
                            uint64_t *d_out_total_bits, int32_t *d_status,
                            void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * ssbh_hash_batch with the same arguments, outputs and error behaviour, but
 * without any device or host allocation.  The hashing plan, tile list and
 * counters live in one fixed library-owned device array of
 * SSBH_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends.
 *  kernel   SSBH_K_VALU, SSBH_K_MFMA_I8 or SSBH_K_MFMA_F4; SSBH_K_AUTO takes
 *           the matrix cores for a shared seed and n_sub >= 64, else VALU
 *           (no tuning table); SSBH_K_FFT gives SSBH_E_UNSUPPORTED (it needs
 *           transform buffers).
 * A request whose plan and tile list exceed the array (roughly
 * 24 n_sub + 16 * tiles bytes; the VALU tiles are about
 * n_sub * (m_cap / rows + 1)) returns SSBH_E_UNSUPPORTED before anything is
 * enqueued.  Every call on one GPU shares the array, which keeps the last
 * call's contents (the path rewrites all it reads): calls that overlap on one
 * GPU -- other streams, other threads, other contexts -- race and must be
 * serialised by the caller.  Schedules forced on ctx apply; ctx's own
 * workspace is not used. */
#define SSBH_NOALLOC_SCRATCH_BYTES (8u << 20)
ssbh_status ssbh_hash_batch_noalloc(ssbh_ctx *ctx, const uint64_t *d_sub,
                                    uint64_t sub_capacity_words,
                                    const uint64_t *d_len,
                                    const uint64_t *d_word_off, uint32_t n_sub,
                                    uint32_t out_rule, uint64_t out_a,
                                    uint64_t out_b, const uint64_t *d_out_len,
                                    const uint64_t *d_seed, uint64_t seed_bits,
                                    uint64_t seed_stride, uint64_t m_cap,
                                    uint32_t kernel, uint64_t *d_out,
                                    uint64_t out_capacity_bits,
                                    uint64_t *d_out_total_bits,
                                    int32_t *d_status, void *stream);

/* Seed bits from a key, on the device: word t of d_seed is output t of the
 * SplitMix64 stream with key seed_key (the generator described at
 * ssbh_sample); bits past seed_bits are zero.  Used for the fresh per-job
 * seeds of the serving loop (a uniform seed, Sec. I). */
ssbh_status ssbh_seed_from_key(ssbh_ctx *ctx, uint64_t seed_key,
                               uint64_t *d_seed, uint64_t seed_bits,
                               void *stream);

/* ------------------------------------------------------ graph pipeline --- */

/* The whole hot path (ssbh_sample then ssbh_hash_batch) on fixed buffers,
 * captured once into a HIP graph and replayed with one launch.  The fields
 * mean what the arguments of the two calls mean; d_in = NULL skips the
 * sampling step (hash-only pipeline over d_sub/d_len/d_word_off as given).
 * Inputs may change between launches; sizes and pointers may not. */
typedef struct {
    const uint64_t *d_in; uint64_t n_bits; uint32_t n_sub; uint32_t mode;
    uint64_t sample_key; const uint32_t *d_assign; uint64_t l_ub;
    uint64_t *d_sub; uint64_t sub_capacity_words;
    uint64_t *d_len; uint64_t *d_word_off;
    uint32_t out_rule; uint64_t out_a, out_b; const uint64_t *d_out_len;
    const uint64_t *d_seed; uint64_t seed_bits; uint64_t seed_stride;
    uint64_t m_cap; uint32_t kernel;
    uint64_t *d_out; uint64_t out_capacity_bits; uint64_t *d_out_total_bits;
    int32_t *d_status;
    const uint64_t *d_keep;  /* sifting flags as in ssbh_sample_sifted, or
                                NULL (no sifting)                           */
} ssbh_pipeline_desc;

typedef struct ssbh_pipeline ssbh_pipeline;

/* Build the pipeline: allocates its own scratch memory (so replays never
 * share scratch with other calls), runs the path once eagerly on a private
 * stream (one-time kernel set-up; the outputs are written), then captures it.
 * Blocks until done. */
ssbh_status ssbh_pipeline_create(ssbh_ctx *ctx, const ssbh_pipeline_desc *desc,
                                 ssbh_pipeline **out);

/* Enqueue one replay of the captured path on `stream` (hipStream_t). */
ssbh_status ssbh_pipeline_launch(ssbh_pipeline *pipe, void *stream);

/* Free the graph and its scratch (waits for the pipeline's replays). */
void ssbh_pipeline_destroy(ssbh_pipeline *pipe);

/* ------------------------------------------------------------ serving --- */

/* One extraction job (the whole method of Sec. III.B on one input block):
 * i.i.d. sampling into n_sub sub-blocks with the abort threshold l_ub,
 * a fresh uniform seed drawn on the device from seed_key, a Toeplitz hash of
 * every sub-block with its OWN seed window (independent hash functions, Sec.
 * III.B step 3) and the concatenation of the outputs.
 *
 * Sizes fixed from the job's parameters (so the result is a function of the
 * job alone):  n_cap = l_ub (if l_ub = 0 the library uses
 * l_ub = ceil(n/n_sub + 8*sqrt(n/n_sub)) + 64);  m_cap = the output rule
 * applied to n_cap;  seed stride S = n_cap + m_cap - 1;  seed length
 * n_sub * S bits (word t of the seed is output t of the SplitMix64 stream
 * keyed by seed_key, as in ssbh_seed_from_key).  The hash kernel is fixed at
 * submission from these sizes: the FFT hash (one transform per sub-block,
 * chunks of at most 48 MiB of transforms) when it pays by the rule stated
 * under ssbh_tune, else the bit-sliced VALU kernel with the schedule the
 * context would choose then; the bits are the same either way. */
typedef struct {
    const uint64_t *in;      /* input bits A^N                               */
    int in_on_device;        /* 1: `in` is device memory, already written
                                when ssbh_submit is called, valid until
                                ssbh_poll returns a terminal status;
                                0: host memory (pinned for an overlapped
                                copy), copied at admission                   */
    uint64_t n_bits;         /* N <= SSBH_MAX_SAMPLE_BITS                    */
    uint32_t n_sub;          /* N_S <= SSBH_MAX_SUB_LDS                      */
    uint64_t sample_key;     /* key of the V_i draws                         */
    uint64_t l_ub;           /* L_S^UB (0 = library default above)           */
    uint32_t out_rule;       /* SSBH_OUT_FIXED or SSBH_OUT_RATIO             */
    uint64_t out_a, out_b;
    uint64_t seed_key;       /* key of the job's fresh seed                  */
    uint64_t *out;           /* result buffer: >= ssbh_job_out_words words   */
    int out_on_device;       /* 1: `out` is device memory; 0: host memory
                                (pinned for an overlapped copy)              */
} ssbh_job;

typedef struct {
    int32_t status;          /* SSBH_OK, SSBH_E_ABORT_OVERSIZE, ...          */
    uint64_t out_bits;       /* total output length sum_j m_j               */
    uint64_t device_bytes;   /* HBM the job held while admitted              */
    double t_submit, t_admit, t_done;   /* seconds, host steady clock        */
} ssbh_result;

/* Words the `out` buffer of a job must hold: ceil((floor(n*a/b) + 64)/64)
 * for the ratio rule, ceil((n_sub*a + 64)/64) for the fixed rule. */
uint64_t ssbh_job_out_words(const ssbh_job *job);

/* Queue a job; never blocks on the device.  Jobs are admitted in FIFO order
 * as soon as a stream slot and enough of the context's HBM budget are free
 * (continuous batching: admitted jobs run concurrently on separate streams).
 * SSBH_E_NOMEM: the job alone exceeds the budget; SSBH_E_INVAL: bad job. */
ssbh_status ssbh_submit(ssbh_ctx *ctx, const ssbh_job *job, uint64_t *job_id);

/* SSBH_PENDING while queued or running; otherwise the job's terminal status
 * (also in res->status), its output already written to job->out, and the id
 * is released.  SSBH_E_UNKNOWN_JOB for an unknown or released id. */
ssbh_status ssbh_poll(ssbh_ctx *ctx, uint64_t job_id, ssbh_result *res);

/* Counters of the serving scheduler: jobs queued, running, finished. */
ssbh_status ssbh_serve_counts(ssbh_ctx *ctx, uint64_t *pending,
                              uint64_t *running, uint64_t *finished);

/* ------------------------------------------------------------- tuning --- */

/* Autotuner: run ssbh_hash_batch on the given (real) arguments once per
 * candidate kernel and schedule (bit-sliced VALU schedules, FFT chunks of
 * 64 .. 256 MiB of transforms (two chunks in flight on two streams), and
 * int8 matrix-core schedules when the seed
 * is shared), `reps` timed runs each with HIP events (after one untimed
 * run; their median counts), and remember the fastest for the shape bucket of these arguments (seed
 * sharing, log2 of n_sub, m_cap and mean sub-block words).  Later calls with
 * kernel = SSBH_K_AUTO in the same bucket use it; without a tuned entry AUTO
 * picks the FFT when n * m_cap >= 1024 L log2 L / k, with n = seed_bits + 1
 * - m_cap (shared seed) or S + 1 - m_cap (seed stride S), L the transform
 * length and k the sub-blocks per transform (4 or 2 for a shared seed, 1
 * with a stride or a single sub-block); else the matrix cores for a shared seed and n_sub >= 64;
 * the VALU kernel in every other case.  Blocks until the stream is idle; d_out holds a valid result
 * afterwards.  If report is non-null, a text table of the timings is written
 * (truncated to report_len bytes). */
ssbh_status ssbh_tune(ssbh_ctx *ctx, const uint64_t *d_sub,
                      uint64_t sub_capacity_words, const uint64_t *d_len,
                      const uint64_t *d_word_off, uint32_t n_sub,
                      uint32_t out_rule, uint64_t out_a, uint64_t out_b,
                      const uint64_t *d_out_len, const uint64_t *d_seed,
                      uint64_t seed_bits, uint64_t seed_stride, uint64_t m_cap,
                      uint64_t *d_out, uint64_t out_capacity_bits,
                      uint64_t *d_out_total_bits, int32_t *d_status,
                      uint32_t reps, char *report, uint64_t report_len,
                      void *stream);

/* The tuned choices, one "bucket=choice" line each (truncated to len). */
ssbh_status ssbh_tune_table(ssbh_ctx *ctx, char *buf, uint64_t len);

/* The kernel and schedule that the last ssbh_hash_batch or ssbh_tune call on
 * this context launched, as "valu:R:waves:chunk_cols:tile_cols" or
 * "mfma:MT:NT:WM:ksplit" (ksplit 0 = automatic) or
 * "fft:chunk:x<sub-blocks per transform>:L<length>", with ":f32" appended
 * when the passes exchange complex floats (empty before the first call;
 * truncated to len). */
ssbh_status ssbh_last_schedule(ssbh_ctx *ctx, char *buf, uint64_t len);

/* Force the schedule of the VALU hash kernel for later calls on this
 * context: r = rows per lane (8, 16 or 32), waves = wavefronts per workgroup
 * (2, 4 or 8; a workgroup tile is 64*r*waves rows), tile_cols = 32-bit column
 * words per tile (0 = whole sub-block), chunk_cols = column words staged in
 * LDS at a time (a multiple of r; 0 = library choice).  0 for r or waves
 * restores the library's choice.  The output bits do not depend on the
 * schedule. */
ssbh_status ssbh_set_schedule(ssbh_ctx *ctx, int r, int waves,
                              uint32_t tile_cols, uint32_t chunk_cols);

/* Force the schedule of the matrix-core kernels (int8 and fp4): mt = 32-row
 * tiles per wavefront, nt = 32-sub-block tiles per wavefront, wm =
 * wavefronts per workgroup (supported: (8,2,4), (4,4,4), (4,2,4), (4,2,8),
 * (8,1,4)); 0s restore the library's choice (two waves per SIMD: (4,2,4) for
 * int8, (4,2,8) for fp4; the tuned choice under SSBH_K_AUTO).  ksplit = K splits per tile (1 .. 64; 0 = chosen so that
 * the tiles fill every compute unit in whole rounds).  The output bits do not
 * depend on any of them. */
ssbh_status ssbh_set_mfma_schedule(ssbh_ctx *ctx, int mt, int nt, int wm,
                                   int ksplit);

/* Per-kernel timing: with on = 1, the synchronous entry points of this
 * context time each launch of their main kernels (k_hist, k_scatter,
 * k_perm_gather, k_toeplitz_valu, k_toeplitz_mfma, k_fft_spectrum, k_fft_cols,
 * k_fft_rows, k_fft_out, k_fft_emit) with a pair of HIP events on the launch
 * stream: k_fft_cols, k_fft_rows (not the spectrum's), k_fft_out and
 * k_fft_emit record them in the launch itself (the kernel's start and end),
 * the others are bracketed by them.  on = 0 stops it and frees the events.
 * Graph pipelines and serving jobs are never timed. */
ssbh_status ssbh_set_timing(ssbh_ctx *ctx, int on);

/* Wait for the recorded launches and write one line per kernel,
 * "name launches total_ms", then forget them (truncated to len). */
ssbh_status ssbh_timing_report(ssbh_ctx *ctx, char *buf, uint64_t len);

/* Placement kernels of the sampling: path 0 = library choice (i.i.d. /
 * explicit: a workgroup of four wavefronts per segment when its LDS tables
 * fit in 64 KiB; permutation: the streaming gather from 2^26 input bits),
 * 1 = the one-wavefront kernels (one wavefront per segment; the direct
 * gather, one random input read per output bit).  The sub-blocks do not
 * depend on it. */
ssbh_status ssbh_set_sample_path(ssbh_ctx *ctx, int path);

/* Force the FFT hash's chunk: transforms per pass (each holds two or four
 * sub-blocks with a shared seed, one with a seed stride, and takes L complex
 * doubles, or complex floats (ssbh_set_fft_storage), of scratch, at most
 * 512 MiB per pass; 0 = library choice).  The output bits do not depend on
 * it. */
ssbh_status ssbh_set_fft_schedule(ssbh_ctx *ctx, uint32_t chunk_pairs);

/* Force how many sub-blocks share each real and imaginary part of an FFT
 * transform with a shared seed: 1 (two per transform), 2 (four: the second
 * scaled by 2^18, needs seed_bits + 1 - m_cap < 2^18 and a transform
 * length of at most 2^20, else the hash returns SSBH_E_UNSUPPORTED), or 0 =
 * library choice (2 when allowed; a single sub-block takes one transform
 * carrying its seed and its bits instead).  For tests and tuning; the output bits
 * do not depend on it. */
ssbh_status ssbh_set_fft_packing(ssbh_ctx *ctx, int per_part);

/* Force the FFT hash's storage of transform data between its passes: 64 =
 * complex doubles, 32 = complex floats (arithmetic stays double), 0 =
 * library choice (floats for one sub-block per transform -- a seed stride
 * S > 0, or a single sub-block without forced packing -- and a transform
 * length of at most 2^18, else doubles).  Floats are allowed only there:
 * elsewhere the hash returns SSBH_E_UNSUPPORTED.  There, rounding both intermediates to
 * float moves each entry s_j * xr_j by less than 5 * 2^-24 * (L + n_j)
 * < 5/32 (L seed bits in the real part, n_j input bits in the imaginary
 * part), below the 1/4 every entry is checked for.  For tests
 * and tuning of the synchronous entry points (serving takes the library
 * choice); the output bits do not depend on it.  bits outside {0, 32, 64}:
 * SSBH_E_INVAL. */
ssbh_status ssbh_set_fft_storage(ssbh_ctx *ctx, int bits);

/* Where the VALU hash kernel reads the 32-bit column words of the sub-blocks
 * from: 0 = staged in LDS with the seed window, 1 = through the scalar data
 * cache straight into scalar registers (one s_load_dwordx8 per 8 words),
 * -1 = library choice.  The output bits do not depend on it. */
ssbh_status ssbh_set_column_path(ssbh_ctx *ctx, int scalar_x);

#ifdef __cplusplus
}
#endif
#endif /* SSBH_H */
