/*
 * CPU oracle for the hashing hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, single-threaded, deliberately unoptimised C.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load this file.
 * The GPU library never includes, links or calls it, and it shares no code,
 * header or table with the GPU path.
 *
 * What it computes and where each definition comes from:
 *   - MD5: RFC 1321, Sec. 3.1-3.5 (padding, length, buffer init, the four
 *     rounds, output).
 *   - SHA-1: FIPS 180-4, Sec. 4.1.1, 4.2.1, 5.1.1, 5.3.1, 6.1.2; direct
 *     hashing with SHA-1 (20-byte segment digests, root over their
 *     concatenation) is the variant of the paper's own measurements
 *     (Sec. 5.2).  The paper's application is StoreGPU's hashing of a
 *     stream of data blocks (Sec. 2.2, Sec. 5.2); it measures SHA1 there,
 *     and MD5 is the primary digest here.
 *   - Direct hashing: the "direct hashing" primitive of Sec. 5.2 (Fig. 6):
 *     digest every fixed-size segment, then the CPU post-processing stage
 *     digests the concatenated segment digests.  Segment size 4 KiB; a short
 *     last segment is hashed as it is; n = 0 gives zero segments and
 *     root = MD5("").
 *   - Content-defined chunking: the content-addressable-storage chunking of
 *     Sec. 2.2 (chunk, then hash each chunk as its identifier).  Window hash
 *     W_i = sum_{k=0}^{47} buf[i-47+k] * B^(47-k) mod 2^64 for i >= 47 (newest
 *     byte has weight B^0); candidate iff (W_i & mask) == 0; chunk rule
 *     walking i = 0..N-1 with len = i+1-s: cut after i when
 *     (len >= min and i is a candidate) or len == max; at end of input emit N
 *     when s < N.  The window is never reset at chunk boundaries.
 *
 * Parity status: every function here is pinned by the CPU test suite
 * (hashlib/OpenSSL and md5sum for MD5, hashlib and sha1sum for SHA-1, brute-force polynomial sums for the
 * window hash, the closed-form all-zero and no-hit cases, chunk-rule
 * invariants, brute-force enumeration of the rule, split invariance).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ MD5 --- */

typedef struct {
    uint32_t st[4];
    uint64_t total;     /* bytes consumed so far */
    uint8_t pend[64];   /* partial block */
    size_t npend;
} omd5_ctx;

static uint32_t T_sine[64];
static int T_ready;

/* RFC 1321 Sec. 3.4: T[i] = floor(4294967296 * |sin(i)|), i = 1..64 radians. */
static void omd5_tables(void)
{
    if (T_ready)
        return;
    for (int i = 0; i < 64; i++)
        T_sine[i] = (uint32_t)floor(fabs(sin((double)(i + 1))) * 4294967296.0);
    T_ready = 1;
}

static uint32_t rotl32(uint32_t x, int s) { return (x << s) | (x >> (32 - s)); }

/* RFC 1321 Sec. 3.4: process one 64-byte block into the state. */
static void omd5_block(uint32_t st[4], const uint8_t blk[64])
{
    static const int S[4][4] = {{7, 12, 17, 22}, {5, 9, 14, 20},
                                {4, 11, 16, 23}, {6, 10, 15, 21}};
    uint32_t X[16];
    for (int j = 0; j < 16; j++) /* little-endian words */
        X[j] = (uint32_t)blk[4 * j] | ((uint32_t)blk[4 * j + 1] << 8) |
               ((uint32_t)blk[4 * j + 2] << 16) | ((uint32_t)blk[4 * j + 3] << 24);
    uint32_t a = st[0], b = st[1], c = st[2], d = st[3];
    for (int i = 0; i < 64; i++) {
        int round = i / 16, j = i % 16, k;
        uint32_t f;
        switch (round) {
        case 0: f = (b & c) | (~b & d); k = j; break;               /* F */
        case 1: f = (b & d) | (c & ~d); k = (1 + 5 * j) % 16; break; /* G */
        case 2: f = b ^ c ^ d;          k = (5 + 3 * j) % 16; break; /* H */
        default: f = c ^ (b | ~d);      k = (7 * j) % 16; break;     /* I */
        }
        uint32_t nb = b + rotl32(a + f + X[k] + T_sine[i], S[round][j % 4]);
        a = d;
        d = c;
        c = b;
        b = nb;
    }
    st[0] += a;
    st[1] += b;
    st[2] += c;
    st[3] += d;
}

static void omd5_init(omd5_ctx *c)
{
    omd5_tables();
    c->st[0] = 0x67452301u; /* RFC 1321 Sec. 3.3 */
    c->st[1] = 0xefcdab89u;
    c->st[2] = 0x98badcfeu;
    c->st[3] = 0x10325476u;
    c->total = 0;
    c->npend = 0;
}

static void omd5_update(omd5_ctx *c, const uint8_t *p, size_t n)
{
    c->total += n;
    while (n) {
        size_t take = 64 - c->npend;
        if (take > n)
            take = n;
        memcpy(c->pend + c->npend, p, take);
        c->npend += take;
        p += take;
        n -= take;
        if (c->npend == 64) {
            omd5_block(c->st, c->pend);
            c->npend = 0;
        }
    }
}

/* RFC 1321 Sec. 3.1-3.2 and 3.5: pad with 0x80 and zeros to 56 mod 64, append
 * the bit length as 64-bit little-endian, emit A,B,C,D little-endian. */
static void omd5_final(omd5_ctx *c, uint8_t out[16])
{
    uint64_t bits = c->total * 8u;
    uint8_t pad = 0x80;
    uint64_t keep = c->total;
    omd5_update(c, &pad, 1);
    uint8_t zero = 0;
    while (c->npend != 56)
        omd5_update(c, &zero, 1);
    uint8_t len[8];
    for (int i = 0; i < 8; i++)
        len[i] = (uint8_t)(bits >> (8 * i));
    omd5_update(c, len, 8);
    c->total = keep;
    for (int w = 0; w < 4; w++)
        for (int i = 0; i < 4; i++)
            out[4 * w + i] = (uint8_t)(c->st[w] >> (8 * i));
}

void oracle_md5(const uint8_t *p, size_t n, uint8_t out[16])
{
    omd5_ctx c;
    omd5_init(&c);
    omd5_update(&c, p, n);
    omd5_final(&c, out);
}

/* ------------------------------------------------------- direct hashing --- */

/* Digest of every `seg`-byte segment (last one may be short), then the digest
 * of the concatenated segment digests.  Returns the segment count. */
size_t oracle_direct(const uint8_t *buf, size_t n, size_t seg,
                     uint8_t *seg_digests, uint8_t root[16])
{
    size_t nseg = (n + seg - 1) / seg;
    for (size_t j = 0; j < nseg; j++) {
        size_t lo = j * seg, hi = lo + seg < n ? lo + seg : n;
        oracle_md5(buf + lo, hi - lo, seg_digests + 16 * j);
    }
    oracle_md5(seg_digests, 16 * nseg, root);
    return nseg;
}

/* MD5 of every buffer of a batch: buffer m is arena[off[m], off[m]+len[m]). */
void oracle_md5_batch(const uint8_t *arena, const uint64_t *off,
                      const uint32_t *len, size_t nbuf, uint8_t *out)
{
    for (size_t m = 0; m < nbuf; m++)
        oracle_md5(arena + off[m], len[m], out + 16 * m);
}

/* MD5 of every chunk buf[ends[k-1], ends[k]) with ends[-1] = 0. */
void oracle_md5_chunks(const uint8_t *buf, const uint64_t *ends, size_t nch,
                       uint8_t *out)
{
    uint64_t lo = 0;
    for (size_t k = 0; k < nch; k++) {
        oracle_md5(buf + lo, ends[k] - lo, out + 16 * k);
        lo = ends[k];
    }
}

/* ----------------------------------------------------------------- SHA-1 --- */
/* FIPS 180-4: Sec. 5.1.1 (padding), 5.3.1 (initial hash value), 4.1.1 (the
 * functions f_t), 4.2.1 (constants K_t), 6.1.2 (the computation: message
 * schedule, working variables, intermediate hash update).  Words are
 * big-endian; the 64-bit message length in bits ends the padded message. */

static uint32_t osha1_f(int t, uint32_t x, uint32_t y, uint32_t z)
{
    if (t < 20)
        return (x & y) ^ (~x & z);           /* Ch */
    if (t < 40)
        return x ^ y ^ z;                    /* Parity */
    if (t < 60)
        return (x & y) ^ (x & z) ^ (y & z);  /* Maj */
    return x ^ y ^ z;                        /* Parity */
}

static uint32_t osha1_k(int t)
{
    if (t < 20)
        return 0x5a827999u;
    if (t < 40)
        return 0x6ed9eba1u;
    if (t < 60)
        return 0x8f1bbcdcu;
    return 0xca62c1d6u;
}

static void osha1_block(uint32_t H[5], const uint8_t blk[64])
{
    uint32_t W[80];
    for (int t = 0; t < 16; t++)
        W[t] = ((uint32_t)blk[4 * t] << 24) | ((uint32_t)blk[4 * t + 1] << 16) |
               ((uint32_t)blk[4 * t + 2] << 8) | (uint32_t)blk[4 * t + 3];
    for (int t = 16; t < 80; t++)
        W[t] = rotl32(W[t - 3] ^ W[t - 8] ^ W[t - 14] ^ W[t - 16], 1);
    uint32_t a = H[0], b = H[1], c = H[2], d = H[3], e = H[4];
    for (int t = 0; t < 80; t++) {
        uint32_t T = rotl32(a, 5) + osha1_f(t, b, c, d) + e + osha1_k(t) + W[t];
        e = d;
        d = c;
        c = rotl32(b, 30);
        b = a;
        a = T;
    }
    H[0] += a;
    H[1] += b;
    H[2] += c;
    H[3] += d;
    H[4] += e;
}

void oracle_sha1(const uint8_t *p, size_t n, uint8_t out[20])
{
    uint32_t H[5] = {0x67452301u, 0xefcdab89u, 0x98badcfeu, 0x10325476u, 0xc3d2e1f0u};
    size_t i = 0;
    for (; i + 64 <= n; i += 64)
        osha1_block(H, p + i);
    /* padding: the remaining bytes, 0x80, zeros, 64-bit big-endian bit count */
    uint8_t last[128];
    size_t r = n - i;
    memset(last, 0, sizeof last);
    memcpy(last, p + i, r);
    last[r] = 0x80;
    size_t total = r + 1 + 8 <= 64 ? 64 : 128;
    uint64_t bits = (uint64_t)n * 8;
    for (int k = 0; k < 8; k++)
        last[total - 1 - k] = (uint8_t)(bits >> (8 * k));
    for (size_t off = 0; off < total; off += 64)
        osha1_block(H, last + off);
    for (int k = 0; k < 5; k++) {
        out[4 * k] = (uint8_t)(H[k] >> 24);
        out[4 * k + 1] = (uint8_t)(H[k] >> 16);
        out[4 * k + 2] = (uint8_t)(H[k] >> 8);
        out[4 * k + 3] = (uint8_t)H[k];
    }
}

/* Direct hashing with SHA-1 (the digest the paper's application measures):
 * SHA-1 of every `seg`-byte segment, then SHA-1 of the concatenated 20-byte
 * segment digests.  Returns the segment count. */
size_t oracle_sha1_direct(const uint8_t *buf, size_t n, size_t seg,
                          uint8_t *seg_digests, uint8_t root[20])
{
    size_t nseg = (n + seg - 1) / seg;
    for (size_t j = 0; j < nseg; j++) {
        size_t lo = j * seg, hi = lo + seg < n ? lo + seg : n;
        oracle_sha1(buf + lo, hi - lo, seg_digests + 20 * j);
    }
    oracle_sha1(seg_digests, 20 * nseg, root);
    return nseg;
}

/* ------------------------------------------------------------ window hash --- */

#define OW 48 /* window width in bytes */

static uint64_t pow64(uint64_t b, unsigned e)
{
    uint64_t r = 1;
    for (unsigned i = 0; i < e; i++)
        r *= b; /* arithmetic mod 2^64 */
    return r;
}

static uint64_t mask_of(int bits)
{
    return bits >= 64 ? ~(uint64_t)0 : (((uint64_t)1 << bits) - 1);
}

/* Window hash at every offset by the rolling identity
 *   W_i = W_{i-1} * B - buf[i-48] * B^48 + buf[i]   (mod 2^64).
 * W[i] for i < 47 (window not yet full) is written as 0. */
void oracle_window_hash(const uint8_t *buf, size_t n, uint64_t base, uint64_t *W)
{
    uint64_t b48 = pow64(base, OW), w = 0;
    for (size_t i = 0; i < n; i++) {
        w = w * base + buf[i];
        if (i >= OW)
            w -= (uint64_t)buf[i - OW] * b48;
        W[i] = i + 1 >= OW ? w : 0;
    }
}

/* The same quantity as the plain 48-term polynomial sum at each offset. */
void oracle_window_hash_brute(const uint8_t *buf, size_t n, uint64_t base,
                              uint64_t *W)
{
    for (size_t i = 0; i < n; i++) {
        if (i + 1 < OW) {
            W[i] = 0;
            continue;
        }
        uint64_t s = 0;
        for (int k = 0; k < OW; k++)
            s += (uint64_t)buf[i - (OW - 1) + k] * pow64(base, (unsigned)(OW - 1 - k));
        W[i] = s;
    }
}

/* Candidate positions {i : i >= 47, (W_i & mask) == 0}, ascending.  Returns
 * the full count; at most `cap` are written. */
size_t oracle_candidates(const uint8_t *buf, size_t n, uint64_t base,
                         int mask_bits, uint64_t *out, size_t cap)
{
    uint64_t b48 = pow64(base, OW), w = 0, m = mask_of(mask_bits);
    size_t cnt = 0;
    for (size_t i = 0; i < n; i++) {
        w = w * base + buf[i];
        if (i >= OW)
            w -= (uint64_t)buf[i - OW] * b48;
        if (i + 1 >= OW && (w & m) == 0) {
            if (cnt < cap)
                out[cnt] = i;
            cnt++;
        }
    }
    return cnt;
}

/* The chunk rule applied to a sorted candidate list, walking every byte
 * position in order.  Returns the chunk count; at most `cap` ends written. */
size_t oracle_select(const uint64_t *cand, size_t k, uint64_t n,
                     uint64_t min_len, uint64_t max_len, uint64_t *ends,
                     size_t cap)
{
    uint64_t s = 0;
    size_t j = 0, cnt = 0;
    for (uint64_t i = 0; i < n; i++) {
        while (j < k && cand[j] < i)
            j++;
        int is_cand = j < k && cand[j] == i;
        uint64_t len = i + 1 - s;
        if ((len >= min_len && is_cand) || len == max_len) {
            if (cnt < cap)
                ends[cnt] = i + 1;
            cnt++;
            s = i + 1;
        }
    }
    if (s < n) {
        if (cnt < cap)
            ends[cnt] = n;
        cnt++;
    }
    return cnt;
}

/* --------------------------------------------------- streaming chunker --- */

/* Carries everything needed to continue across feed() calls: position, chunk
 * start, window bytes, rolling value and the current chunk's MD5 state. */
typedef struct {
    uint64_t base, b48, mask, min_len, max_len;
    uint64_t pos;   /* bytes consumed so far */
    uint64_t start; /* start offset of the open chunk */
    uint64_t w;
    uint8_t ring[OW];
    omd5_ctx md;
} oracle_cdc;

oracle_cdc *oracle_cdc_new(uint64_t base, int mask_bits, uint64_t min_len,
                           uint64_t max_len)
{
    oracle_cdc *c = (oracle_cdc *)calloc(1, sizeof(*c));
    if (!c)
        return NULL;
    c->base = base;
    c->b48 = pow64(base, OW);
    c->mask = mask_of(mask_bits);
    c->min_len = min_len;
    c->max_len = max_len;
    omd5_init(&c->md);
    return c;
}

void oracle_cdc_free(oracle_cdc *c) { free(c); }

/* Consume p[0..n); every chunk that closes is reported as its end offset and
 * digest.  Returns how many closed (at most `cap` are written). */
size_t oracle_cdc_feed(oracle_cdc *c, const uint8_t *p, size_t n,
                       uint64_t *ends, uint8_t *digests, size_t cap)
{
    size_t cnt = 0, hashed_from = 0;
    for (size_t t = 0; t < n; t++) {
        uint64_t i = c->pos++;
        uint8_t b = p[t];
        c->w = c->w * c->base + b;
        if (i >= OW)
            c->w -= (uint64_t)c->ring[i % OW] * c->b48;
        c->ring[i % OW] = b;
        int is_cand = i + 1 >= OW && (c->w & c->mask) == 0;
        uint64_t len = i + 1 - c->start;
        if ((len >= c->min_len && is_cand) || len == c->max_len) {
            omd5_update(&c->md, p + hashed_from, t + 1 - hashed_from);
            hashed_from = t + 1;
            if (cnt < cap) {
                ends[cnt] = i + 1;
                omd5_final(&c->md, digests + 16 * cnt);
            }
            cnt++;
            omd5_init(&c->md);
            c->start = i + 1;
        }
    }
    omd5_update(&c->md, p + hashed_from, n - hashed_from);
    return cnt;
}

/* End of input: close the open chunk if it is non-empty. */
size_t oracle_cdc_finish(oracle_cdc *c, uint64_t *ends, uint8_t *digests,
                         size_t cap)
{
    if (c->start >= c->pos)
        return 0;
    if (cap >= 1) {
        ends[0] = c->pos;
        omd5_final(&c->md, digests);
    }
    c->start = c->pos;
    omd5_init(&c->md);
    return 1;
}
