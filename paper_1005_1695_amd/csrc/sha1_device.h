// Device-side SHA-1 for gfx950 (FIPS 180-4, Sec. 6.1.2).
//
// As for MD5, one lane owns one message and walks its 64-byte blocks
// serially.  The compression is fully unrolled: the 16-word message schedule
// window stays in VGPRs and is extended in place (W[t] for t >= 16 from
// W[t-3], W[t-8], W[t-14], W[t-16]); Ch, Maj and the three-input parity map to
// one v_bitop3_b32 (or v_bfi_b32) each, the rotates to v_alignbit_b32, the
// five-term sum to two three-input adds: about 600 VALU ops per block.
// Message words are big-endian: the little-endian dwords the loads return are
// byte-swapped (v_perm_b32).
//
// Readability contract (as for the MD5 loaders): the bytes of a message
// [p, p+len) may be read in whole aligned dwords / 16-byte vectors, so the
// buffer must be readable up to the next 16-byte boundary after p+len.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crystal {

__device__ __forceinline__ uint32_t sha1_rotl(uint32_t x, int s)
{
    return __builtin_rotateleft32(x, s);
}

// Three-input exclusive or in one v_bitop3_b32 (truth table 0x96); the
// compiler does not form it from two-input xors by itself.
__device__ __forceinline__ uint32_t sha1_xor3(uint32_t x, uint32_t y, uint32_t z)
{
    return __builtin_amdgcn_bitop3_b32(x, y, z, 0x96);
}

// One step t of Sec. 6.1.2 with round function FN and constant K.
#define S1_CH(b, c, d) (((b) & (c)) | (~(b) & (d)))
#define S1_PAR(b, c, d) sha1_xor3((b), (c), (d))
#define S1_MAJ(b, c, d) (((b) & (c)) | ((b) & (d)) | ((c) & (d)))
#define S1_STEP(FN, K, a, b, c, d, e, w)                                                \
    do {                                                                               \
        (e) += sha1_rotl((a), 5) + FN((b), (c), (d)) + (K) + (w);                      \
        (b) = sha1_rotl((b), 30);                                                      \
    } while (0)

// Schedule word t (t >= 16) written over w[t mod 16].
#define S1_SCHED(w, t)                                                                 \
    ((w)[(t) & 15] = sha1_rotl(sha1_xor3((w)[((t) - 3) & 15], (w)[((t) - 8) & 15],       \
                                         (w)[((t) - 14) & 15]) ^ (w)[(t) & 15],          \
                               1))

// One 64-byte block; x[] holds its 16 big-endian message words.  The working
// variables rotate by renaming: step t uses (a,b,c,d,e) = v[(5-t) mod 5 ...],
// so no register moves are needed.
__device__ __forceinline__ void sha1_compress(uint32_t H[5], const uint32_t x[16])
{
    uint32_t w[16];
#pragma unroll
    for (int k = 0; k < 16; k++)
        w[k] = x[k];
    uint32_t v[5] = {H[0], H[1], H[2], H[3], H[4]};
#pragma unroll
    for (int t = 0; t < 80; t++) {
        uint32_t &a = v[(100 - t) % 5], &b = v[(101 - t) % 5], &c = v[(102 - t) % 5],
                 &d = v[(103 - t) % 5], &e = v[(104 - t) % 5];
        uint32_t wt;
        if (t < 16)
            wt = w[t];
        else
            wt = S1_SCHED(w, t);
        if (t < 20)
            S1_STEP(S1_CH, 0x5a827999u, a, b, c, d, e, wt);
        else if (t < 40)
            S1_STEP(S1_PAR, 0x6ed9eba1u, a, b, c, d, e, wt);
        else if (t < 60)
            S1_STEP(S1_MAJ, 0x8f1bbcdcu, a, b, c, d, e, wt);
        else
            S1_STEP(S1_PAR, 0xca62c1d6u, a, b, c, d, e, wt);
    }
    // after 80 steps (a multiple of 5) the names line up with v[0..4] again
#pragma unroll
    for (int k = 0; k < 5; k++)
        H[k] += v[k];
}

__device__ __forceinline__ void sha1_init(uint32_t H[5])
{
    H[0] = 0x67452301u;
    H[1] = 0xefcdab89u;
    H[2] = 0x98badcfeu;
    H[3] = 0x10325476u;
    H[4] = 0xc3d2e1f0u;
}

// Final block(s): w[] holds the message's last r (< 64) bytes as the raw
// little-endian dwords the loads returned (any content beyond byte r);
// appends 0x80, zero fill and the 64-bit big-endian bit length.
__device__ __forceinline__ void sha1_finish(uint32_t H[5], const uint32_t w[16], uint32_t r,
                                            uint64_t total_len)
{
    uint32_t x[16];
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const int rem = (int)r - 4 * k;
        const uint32_t keep =
            rem >= 4 ? 0xffffffffu : (rem > 0 ? ((1u << (8 * rem)) - 1u) : 0u);
        const uint32_t pad = (rem >= 0 && rem < 4) ? (0x80u << (8 * rem)) : 0u;
        x[k] = __builtin_bswap32((w[k] & keep) | pad);
    }
    const uint64_t bits = total_len << 3;
    if (r < 56) {
        x[14] = (uint32_t)(bits >> 32);
        x[15] = (uint32_t)bits;
        sha1_compress(H, x);
    } else {
        sha1_compress(H, x);
#pragma unroll
        for (int k = 0; k < 14; k++)
            x[k] = 0;
        x[14] = (uint32_t)(bits >> 32);
        x[15] = (uint32_t)bits;
        sha1_compress(H, x);
    }
}

__device__ __forceinline__ void sha1_block_le(uint32_t H[5], const uint4 &v0, const uint4 &v1,
                                              const uint4 &v2, const uint4 &v3)
{
    const uint32_t x[16] = {
        __builtin_bswap32(v0.x), __builtin_bswap32(v0.y), __builtin_bswap32(v0.z),
        __builtin_bswap32(v0.w), __builtin_bswap32(v1.x), __builtin_bswap32(v1.y),
        __builtin_bswap32(v1.z), __builtin_bswap32(v1.w), __builtin_bswap32(v2.x),
        __builtin_bswap32(v2.y), __builtin_bswap32(v2.z), __builtin_bswap32(v2.w),
        __builtin_bswap32(v3.x), __builtin_bswap32(v3.y), __builtin_bswap32(v3.z),
        __builtin_bswap32(v3.w)};
    sha1_compress(H, x);
}

// SHA-1 of a message that starts on a 16-byte boundary.  Blocks are read as
// 16-byte vectors, double-buffered one block ahead: the next block's loads
// are issued (at an index clamped inside the message, so unconditionally)
// before the current one is compressed.
__device__ __forceinline__ void sha1_message_a16(const uint8_t *__restrict__ p, uint64_t len,
                                                 uint32_t H[5])
{
    sha1_init(H);
    const uint4 *q = reinterpret_cast<const uint4 *>(p);
    const uint64_t nb = len >> 6;
    if (nb) {
        uint4 a0 = q[0], a1 = q[1], a2 = q[2], a3 = q[3];
        uint64_t b = 0;
        for (; b + 1 < nb; b += 2) {
            const uint4 *r = q + 4 * (b + 1);
            uint4 b0 = r[0], b1 = r[1], b2 = r[2], b3 = r[3];
            __builtin_amdgcn_sched_barrier(0);
            sha1_block_le(H, a0, a1, a2, a3);
            __builtin_amdgcn_sched_barrier(0);
            const uint64_t nx = b + 2 < nb ? b + 2 : nb - 1;
            const uint4 *s = q + 4 * nx;
            a0 = s[0];
            a1 = s[1];
            a2 = s[2];
            a3 = s[3];
            __builtin_amdgcn_sched_barrier(0);
            sha1_block_le(H, b0, b1, b2, b3);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (b < nb) // odd block count: a holds block nb - 1
            sha1_block_le(H, a0, a1, a2, a3);
    }
    const uint32_t rb = (uint32_t)(len & 63);
    const uint4 *t = q + 4 * nb;
    const uint4 z = make_uint4(0, 0, 0, 0);
    const uint4 t0 = rb > 0 ? t[0] : z;
    const uint4 t1 = rb > 16 ? t[1] : z;
    const uint4 t2 = rb > 32 ? t[2] : z;
    const uint4 t3 = rb > 48 ? t[3] : z;
    const uint32_t w[16] = {t0.x, t0.y, t0.z, t0.w, t1.x, t1.y, t1.z, t1.w,
                            t2.x, t2.y, t2.z, t2.w, t3.x, t3.y, t3.z, t3.w};
    sha1_finish(H, w, rb, len);
}

// SHA-1 of a message at any byte address: each block is read as 17 aligned
// dwords starting at the dword that holds its first byte and realigned with
// v_alignbyte_b32 (the extra dword's index is clamped to the dword holding
// the message's last byte, so it stays readable).
__device__ __forceinline__ void sha1_message_any(const uint8_t *__restrict__ p, uint64_t len,
                                                 uint32_t H[5])
{
    sha1_init(H);
    const uint32_t bs = (uint32_t)((uintptr_t)p & 3);
    const uint32_t *d = reinterpret_cast<const uint32_t *>(p - bs);
    const uint64_t nb = len >> 6;
    const uint64_t dmax = len ? (bs + len - 1) >> 2 : 0;
    for (uint64_t b = 0; b < nb; ++b) {
        uint32_t u[17];
#pragma unroll
        for (int k = 0; k < 16; k++)
            u[k] = d[16 * b + k];
        const uint64_t e16 = 16 * b + 16 < dmax ? 16 * b + 16 : dmax;
        u[16] = d[e16];
        uint32_t x[16];
#pragma unroll
        for (int k = 0; k < 16; k++)
            x[k] = __builtin_bswap32(__builtin_amdgcn_alignbyte(u[k + 1], u[k], bs));
        sha1_compress(H, x);
    }
    const uint32_t rb = (uint32_t)(len & 63);
    const uint32_t *t = d + 16 * nb;
    const uint32_t span = rb ? (bs + rb + 3) >> 2 : 0u;
    uint32_t u[17];
#pragma unroll
    for (int k = 0; k < 17; k++)
        u[k] = (uint32_t)k < span ? t[k] : 0u;
    uint32_t w[16];
#pragma unroll
    for (int k = 0; k < 16; k++)
        w[k] = __builtin_amdgcn_alignbyte(u[k + 1], u[k], bs);
    sha1_finish(H, w, rb, len);
}

// The 20-byte digest (H0..H4 big-endian) at a 4-byte-aligned address.
__device__ __forceinline__ void sha1_store(uint8_t *__restrict__ out, const uint32_t H[5])
{
    uint32_t *o = reinterpret_cast<uint32_t *>(out);
#pragma unroll
    for (int k = 0; k < 5; k++)
        o[k] = __builtin_bswap32(H[k]);
}

#undef S1_CH
#undef S1_PAR
#undef S1_MAJ
#undef S1_STEP
#undef S1_SCHED

} // namespace crystal
