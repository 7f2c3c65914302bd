/*
 * Plain CPU oracle for sampled sub-block hashing.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
 * CPU-baseline leg of the benchmark may load this file's library.  It shares
 * no code, header, table or constant generator with the GPU library: every
 * routine here is written out directly from the paper's definitions.
 *
 * What it computes (paper references by section / equation):
 *   - Toeplitz hashing, Sec. I: K = T . A' over GF(2), T diagonal-constant and
 *     built from a uniform seed; rows = output length, columns = input length.
 *     Convention (the paper fixes no bit placement):
 *         T_j[r][c] = s[j*S + c - r + M - 1],   0 <= r < m_j, 0 <= c < n_j,
 *     S = seed stride between sub-blocks (0 = one shared seed), M = row cap
 *     (M >= every m_j).  With one block and M = m this is T[r][c] = s[c-r+m-1]:
 *     row r is the seed window starting at bit m-1-r.
 *   - Sampling, Sec. III.B step 1: every round i gets a uniform V_i in
 *     [0, N_S) (0-based); sub-block j holds the bits with V_i = j, in
 *     ascending i (App. B: the sub-block-k view of round i is A'_i when
 *     V_i = k and empty otherwise, so the sub-block is the ordered list of the
 *     kept rounds).
 *   - Abort threshold, Sec. III.B step 2 / Sec. III.D: abort when some
 *     sub-block is longer than L_S^UB (done by the caller from the lengths).
 *   - Extraction per sub-block and concatenation, Sec. III.B steps 3-4:
 *     K = K_0 || K_1 || ... with K_j at bit offset sum_{k<j} m_k.
 *
 * Random numbers: the i.i.d. sampling variables come from SplitMix64
 * (G. Steele, D. Lea, C. Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014; the reference "splitmix64" of S. Vigna): the t-th
 * output (t = 0, 1, ...) for a 64-bit key is mix(key + (t+1)*0x9E3779B97F4A7C15)
 * with the variant-13 finaliser.  Round i uses the low 32 bits of output
 * floor(i/2) when i is even and the high 32 bits when i is odd, and
 * V_i = floor(u_i * N_S / 2^32).
 *
 * Bits: bit k of a string is (w[k >> 6] >> (k & 63)) & 1.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ull

static inline int get_bit(const uint64_t *w, uint64_t k) {
    return (int)((w[k >> 6] >> (k & 63)) & 1ull);
}

static inline void put_bit(uint64_t *w, uint64_t k, int b) {
    if (b) w[k >> 6] |= 1ull << (k & 63);
    else   w[k >> 6] &= ~(1ull << (k & 63));
}

/* ---------------------------------------------------------------- PRNG --- */

uint64_t ssbo_splitmix64(uint64_t key, uint64_t t) {
    uint64_t z = key + (t + 1ull) * GAMMA;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Sequential form of the same stream (state += gamma; output mix(state)),
 * kept separate so the tests can check the counter form against it. */
void ssbo_splitmix64_seq(uint64_t key, uint64_t count, uint64_t *out) {
    uint64_t state = key;
    for (uint64_t t = 0; t < count; ++t) {
        state += GAMMA;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        out[t] = z ^ (z >> 31);
    }
}

/* V_i for one round (Sec. III.B step 1, 0-based). */
uint32_t ssbo_draw_v(uint64_t key, uint64_t i, uint32_t n_sub) {
    uint64_t r = ssbo_splitmix64(key, i >> 1);
    uint32_t u = (i & 1ull) ? (uint32_t)(r >> 32) : (uint32_t)r;
    return (uint32_t)(((uint64_t)u * (uint64_t)n_sub) >> 32);
}

void ssbo_assign_iid(uint64_t n, uint32_t n_sub, uint64_t key, uint32_t *v) {
    for (uint64_t i = 0; i < n; ++i) v[i] = ssbo_draw_v(key, i, n_sub);
}

/* Seed bits drawn from a key: word t of the seed is output t of the stream. */
void ssbo_seed_from_key(uint64_t key, uint64_t n_bits, uint64_t *seed) {
    uint64_t nw = (n_bits + 63) / 64;
    for (uint64_t t = 0; t < nw; ++t) seed[t] = ssbo_splitmix64(key, t);
    if (n_bits & 63) seed[nw - 1] &= (1ull << (n_bits & 63)) - 1ull;
}

/* ------------------------------------------------------------ sampling --- */

/* Sub-block lengths n_j and 64-bit word offsets W_j = sum_{k<j} ceil(n_k/64). */
void ssbo_lengths(const uint32_t *v, uint64_t n, uint32_t n_sub,
                  uint64_t *len, uint64_t *word_off) {
    memset(len, 0, sizeof(uint64_t) * n_sub);
    for (uint64_t i = 0; i < n; ++i) len[v[i]] += 1;
    uint64_t acc = 0;
    for (uint32_t j = 0; j < n_sub; ++j) {
        word_off[j] = acc;
        acc += (len[j] + 63) / 64;
    }
}

/* Divide A by the assignment V: sub-block j = (A_i : V_i = j) in ascending i,
 * starting at bit 64*W_j of `sub`.  Returns 0, or -1 on a bad V or a too
 * small output buffer. */
int ssbo_partition(const uint64_t *a, uint64_t n, const uint32_t *v,
                   uint32_t n_sub, uint64_t *sub, uint64_t sub_cap_words,
                   uint64_t *len, uint64_t *word_off) {
    for (uint64_t i = 0; i < n; ++i)
        if (v[i] >= n_sub) return -1;
    ssbo_lengths(v, n, n_sub, len, word_off);
    uint64_t need = n_sub ? word_off[n_sub - 1] + (len[n_sub - 1] + 63) / 64 : 0;
    if (need > sub_cap_words) return -1;
    memset(sub, 0, sizeof(uint64_t) * need);
    uint64_t *cursor = (uint64_t *)calloc(n_sub ? n_sub : 1, sizeof(uint64_t));
    if (!cursor) return -1;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t j = v[i];
        put_bit(sub, 64ull * word_off[j] + cursor[j], get_bit(a, i));
        cursor[j] += 1;
    }
    free(cursor);
    return 0;
}

/* Sifting inside every sub-block (Sec. III.B step 2): sub-block j of the
 * data and sub-block j of the keep flags (both divided by the same V) are
 * walked together, and only the bits whose flag is 1 are kept, in order.
 * Output sub-block j starts at word out_off[j] = sum_{k<j} ceil(out_len[k]/64).
 * Returns 0, or -1 when the output buffer is too small. */
int ssbo_sift(const uint64_t *sub, const uint64_t *keep_sub,
              const uint64_t *len, const uint64_t *word_off, uint32_t n_sub,
              uint64_t *out, uint64_t out_cap_words, uint64_t *out_len,
              uint64_t *out_off) {
    for (uint32_t j = 0; j < n_sub; ++j) {
        uint64_t c = 0;
        for (uint64_t k = 0; k < len[j]; ++k)
            c += get_bit(keep_sub, 64ull * word_off[j] + k);
        out_len[j] = c;
    }
    uint64_t acc = 0;
    for (uint32_t j = 0; j < n_sub; ++j) {
        out_off[j] = acc;
        acc += (out_len[j] + 63) / 64;
    }
    if (acc > out_cap_words) return -1;
    memset(out, 0, sizeof(uint64_t) * acc);
    for (uint32_t j = 0; j < n_sub; ++j) {
        uint64_t pos = 0;
        for (uint64_t k = 0; k < len[j]; ++k) {
            const uint64_t b = 64ull * word_off[j] + k;
            if (get_bit(keep_sub, b)) {
                put_bit(out, 64ull * out_off[j] + pos, get_bit(sub, b));
                pos += 1;
            }
        }
    }
    return 0;
}

/* Keyed permutation of 0..n-1 (the permute-split sampling of the small and
 * contraction workloads; not in the paper, which draws V_i i.i.d.).
 * Durstenfeld's form of the Fisher-Yates shuffle (R. Durstenfeld, CACM 7(7),
 * 1964, Algorithm 235): start from the identity and, for i = n-1 down to 1,
 * exchange entries i and j_i, where j_i is uniform in [0, i].  Here j_i is
 * the high word of the 128-bit product r_t * (i + 1), r_t = output
 * t = n-1-i of the SplitMix64 stream of `key` (Lemire's multiply-shift map
 * without the rejection step; its bias is below (i+1)/2^64).  Writes perm[],
 * returns 0, or -1 for n > 2^32. */
uint64_t ssbo_shuffle_choice(uint64_t key, uint64_t n, uint64_t i) {
    uint64_t r = ssbo_splitmix64(key, n - 1 - i);
    return (uint64_t)(((unsigned __int128)r * (i + 1)) >> 64);
}

int ssbo_permutation(uint64_t key, uint64_t n, uint32_t *perm) {
    if (n > (1ull << 32)) return -1;
    for (uint64_t k = 0; k < n; ++k) perm[k] = (uint32_t)k;
    for (uint64_t i = n; i-- > 1;) {
        uint64_t j = ssbo_shuffle_choice(key, n, i);
        uint32_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }
    return 0;
}

/* Permutation then contiguous split: B[k] = A[perm[k]], sub-block j is
 * B[jL, (j+1)L) with L = n / n_sub, starting at word j*ceil(L/64).
 * Returns -1 when n_sub does not divide n or perm is out of range. */
int ssbo_permute_split(const uint64_t *a, uint64_t n, const uint32_t *perm,
                       uint32_t n_sub, uint64_t *sub, uint64_t *len,
                       uint64_t *word_off) {
    if (n_sub == 0 || n % n_sub) return -1;
    uint64_t L = n / n_sub, wl = (L + 63) / 64;
    memset(sub, 0, sizeof(uint64_t) * wl * n_sub);
    for (uint32_t j = 0; j < n_sub; ++j) {
        len[j] = L;
        word_off[j] = (uint64_t)j * wl;
        for (uint64_t c = 0; c < L; ++c) {
            uint64_t k = (uint64_t)j * L + c;
            if (perm[k] >= n) return -1;
            put_bit(sub, 64ull * word_off[j] + c, get_bit(a, perm[k]));
        }
    }
    return 0;
}

/* Output lengths: rule 0 = fixed m_j = a (the l~ of Sec. III.B step 3);
 * rule 1 = floor(n_j * a / b) in exact integer arithmetic. */
void ssbo_out_lengths(const uint64_t *len, uint32_t n_sub, int rule,
                      uint64_t a, uint64_t b, uint64_t *out_len) {
    for (uint32_t j = 0; j < n_sub; ++j) {
        if (rule == 0) out_len[j] = a;
        else {
            unsigned __int128 p = (unsigned __int128)len[j] * a;
            out_len[j] = (uint64_t)(p / b);
        }
    }
}

/* ------------------------------------------------------------ Toeplitz --- */

/* One output bit, straight from the definition:
 *   K[r] = XOR_{c<n} s[base + c - r + cap - 1] AND x[c]. */
int ssbo_toeplitz_row(const uint64_t *x, uint64_t n, const uint64_t *seed,
                      uint64_t base, uint64_t cap, uint64_t r) {
    int acc = 0;
    for (uint64_t c = 0; c < n; ++c)
        acc ^= get_bit(seed, base + c - r + cap - 1) & get_bit(x, c);
    return acc;
}

static int seed_ok(uint64_t n, uint64_t m, uint64_t base, uint64_t cap,
                   uint64_t seed_bits) {
    if (m > cap) return 0;
    if (n == 0 || m == 0) return 1;
    return base + n - 1 + cap - 1 < seed_bits;
}

/* Level 0: bit by bit.  Writes m bits at bit offset out_bit0 of `out`. */
int ssbo_toeplitz_bits(const uint64_t *x, uint64_t n, const uint64_t *seed,
                       uint64_t seed_bits, uint64_t base, uint64_t cap,
                       uint64_t m, uint64_t *out, uint64_t out_bit0) {
    if (!seed_ok(n, m, base, cap, seed_bits)) return -1;
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < (int64_t)m; ++r) {
        int b = ssbo_toeplitz_row(x, n, seed, base, cap, (uint64_t)r);
        if (b) {
            uint64_t k = out_bit0 + (uint64_t)r;
            #pragma omp atomic
            out[k >> 6] |= 1ull << (k & 63);
        }
    }
    return 0;
}

/* 64 seed bits starting at bit `pos` (bits past seed_bits read as 0). */
static inline uint64_t seed_word_at(const uint64_t *seed, uint64_t seed_bits,
                                    uint64_t pos) {
    uint64_t w = pos >> 6, sh = pos & 63, nw = (seed_bits + 63) / 64;
    uint64_t lo = w < nw ? seed[w] : 0ull;
    if (sh == 0) return lo;
    uint64_t hi = (w + 1) < nw ? seed[w + 1] : 0ull;
    return (lo >> sh) | (hi << (64 - sh));
}

/* Level 1: row r is the seed window starting at bit base + cap - 1 - r; AND it
 * with x word by word and take the parity of the population count. */
int ssbo_toeplitz_rowwin(const uint64_t *x, uint64_t n, const uint64_t *seed,
                         uint64_t seed_bits, uint64_t base, uint64_t cap,
                         uint64_t r) {
    uint64_t start = base + cap - 1 - r, nw = (n + 63) / 64, acc = 0;
    for (uint64_t w = 0; w < nw; ++w) {
        uint64_t xw = x[w];
        if (w == nw - 1 && (n & 63)) xw &= (1ull << (n & 63)) - 1ull;
        acc ^= seed_word_at(seed, seed_bits, start + 64 * w) & xw;
    }
    return __builtin_popcountll(acc) & 1;
}

int ssbo_toeplitz_window(const uint64_t *x, uint64_t n, const uint64_t *seed,
                         uint64_t seed_bits, uint64_t base, uint64_t cap,
                         uint64_t m, uint64_t *out, uint64_t out_bit0) {
    if (!seed_ok(n, m, base, cap, seed_bits)) return -1;
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < (int64_t)m; ++r) {
        int b = ssbo_toeplitz_rowwin(x, n, seed, seed_bits, base, cap,
                                     (uint64_t)r);
        if (b) {
            uint64_t k = out_bit0 + (uint64_t)r;
            #pragma omp atomic
            out[k >> 6] |= 1ull << (k & 63);
        }
    }
    return 0;
}

/* Every sub-block hashed with its own T_j (seed offset j*stride) and the
 * outputs concatenated (Sec. III.B steps 3-4).  `out` must hold out_cap_bits
 * bits; it is cleared first.  level 0 = bit by bit, 1 = row windows.
 * Returns the total output length, or -1 on bad arguments. */
int64_t ssbo_hash_batch(const uint64_t *sub, const uint64_t *len,
                        const uint64_t *word_off, uint32_t n_sub,
                        const uint64_t *out_len, const uint64_t *seed,
                        uint64_t seed_bits, uint64_t stride, uint64_t cap,
                        uint64_t *out, uint64_t out_cap_bits, int level) {
    uint64_t total = 0;
    for (uint32_t j = 0; j < n_sub; ++j) total += out_len[j];
    if (total > out_cap_bits) return -1;
    memset(out, 0, sizeof(uint64_t) * ((out_cap_bits + 63) / 64));
    uint64_t off = 0;
    for (uint32_t j = 0; j < n_sub; ++j) {
        const uint64_t *x = sub + word_off[j];
        uint64_t base = (uint64_t)j * stride;
        int rc = level == 0
            ? ssbo_toeplitz_bits(x, len[j], seed, seed_bits, base, cap,
                                 out_len[j], out, off)
            : ssbo_toeplitz_window(x, len[j], seed, seed_bits, base, cap,
                                   out_len[j], out, off);
        if (rc) return -1;
        off += out_len[j];
    }
    return (int64_t)total;
}

/* Threads the OpenMP loops above use (reported with CPU timings). */
#ifdef _OPENMP
#include <omp.h>
int ssbo_threads(void) { return omp_get_max_threads(); }
void ssbo_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
#else
int ssbo_threads(void) { return 1; }
void ssbo_set_threads(int n) { (void)n; }
#endif
