// Device-side MD5 for gfx950 (RFC 1321).
//
// One lane owns one message and walks its 64-byte blocks serially: MD5 is a
// single dependency chain per message, so parallelism comes only from running
// many messages side by side (one per lane).  The compression is fully
// unrolled so the 16 message words and the 4 state words stay in VGPRs; the
// round functions are written so the compiler selects v_bfi_b32 (F, G),
// v_xor3-style chains (H), v_add3_u32 for the three-input sums and
// v_alignbit_b32 for the rotates.
//
// Readability contract of every loader here: the bytes of a message
// [p, p+len) may be read in whole aligned dwords/16-byte vectors, so the
// buffer must be readable up to the next 16-byte boundary after p+len.
// Bytes beyond the message are loaded but never enter the digest.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crystal {

typedef uint32_t u32x4a4 __attribute__((ext_vector_type(4), aligned(4)));

__device__ __forceinline__ uint32_t md5_rotl(uint32_t x, int s)
{
    return __builtin_rotateleft32(x, s);
}

#define CR_F(b, c, d) ((d) ^ ((b) & ((c) ^ (d))))
#define CR_G(b, c, d) ((c) ^ ((d) & ((b) ^ (c))))
#define CR_H(b, c, d) ((b) ^ (c) ^ (d))
#define CR_I(b, c, d) ((c) ^ ((b) | ~(d)))
#define CR_STEP(FN, a, b, c, d, x, t, s) \
    (a) = (b) + md5_rotl((a) + FN((b), (c), (d)) + (x) + (t), (s))

// One 64-byte block; x[] holds its 16 little-endian words.
__device__ __forceinline__ void md5_compress(uint32_t st[4], const uint32_t x[16])
{
    uint32_t a = st[0], b = st[1], c = st[2], d = st[3];
    // round 1: word k = j
    CR_STEP(CR_F, a, b, c, d, x[0], 0xd76aa478u, 7);
    CR_STEP(CR_F, d, a, b, c, x[1], 0xe8c7b756u, 12);
    CR_STEP(CR_F, c, d, a, b, x[2], 0x242070dbu, 17);
    CR_STEP(CR_F, b, c, d, a, x[3], 0xc1bdceeeu, 22);
    CR_STEP(CR_F, a, b, c, d, x[4], 0xf57c0fafu, 7);
    CR_STEP(CR_F, d, a, b, c, x[5], 0x4787c62au, 12);
    CR_STEP(CR_F, c, d, a, b, x[6], 0xa8304613u, 17);
    CR_STEP(CR_F, b, c, d, a, x[7], 0xfd469501u, 22);
    CR_STEP(CR_F, a, b, c, d, x[8], 0x698098d8u, 7);
    CR_STEP(CR_F, d, a, b, c, x[9], 0x8b44f7afu, 12);
    CR_STEP(CR_F, c, d, a, b, x[10], 0xffff5bb1u, 17);
    CR_STEP(CR_F, b, c, d, a, x[11], 0x895cd7beu, 22);
    CR_STEP(CR_F, a, b, c, d, x[12], 0x6b901122u, 7);
    CR_STEP(CR_F, d, a, b, c, x[13], 0xfd987193u, 12);
    CR_STEP(CR_F, c, d, a, b, x[14], 0xa679438eu, 17);
    CR_STEP(CR_F, b, c, d, a, x[15], 0x49b40821u, 22);
    // round 2: word k = (1 + 5j) mod 16
    CR_STEP(CR_G, a, b, c, d, x[1], 0xf61e2562u, 5);
    CR_STEP(CR_G, d, a, b, c, x[6], 0xc040b340u, 9);
    CR_STEP(CR_G, c, d, a, b, x[11], 0x265e5a51u, 14);
    CR_STEP(CR_G, b, c, d, a, x[0], 0xe9b6c7aau, 20);
    CR_STEP(CR_G, a, b, c, d, x[5], 0xd62f105du, 5);
    CR_STEP(CR_G, d, a, b, c, x[10], 0x02441453u, 9);
    CR_STEP(CR_G, c, d, a, b, x[15], 0xd8a1e681u, 14);
    CR_STEP(CR_G, b, c, d, a, x[4], 0xe7d3fbc8u, 20);
    CR_STEP(CR_G, a, b, c, d, x[9], 0x21e1cde6u, 5);
    CR_STEP(CR_G, d, a, b, c, x[14], 0xc33707d6u, 9);
    CR_STEP(CR_G, c, d, a, b, x[3], 0xf4d50d87u, 14);
    CR_STEP(CR_G, b, c, d, a, x[8], 0x455a14edu, 20);
    CR_STEP(CR_G, a, b, c, d, x[13], 0xa9e3e905u, 5);
    CR_STEP(CR_G, d, a, b, c, x[2], 0xfcefa3f8u, 9);
    CR_STEP(CR_G, c, d, a, b, x[7], 0x676f02d9u, 14);
    CR_STEP(CR_G, b, c, d, a, x[12], 0x8d2a4c8au, 20);
    // round 3: word k = (5 + 3j) mod 16
    CR_STEP(CR_H, a, b, c, d, x[5], 0xfffa3942u, 4);
    CR_STEP(CR_H, d, a, b, c, x[8], 0x8771f681u, 11);
    CR_STEP(CR_H, c, d, a, b, x[11], 0x6d9d6122u, 16);
    CR_STEP(CR_H, b, c, d, a, x[14], 0xfde5380cu, 23);
    CR_STEP(CR_H, a, b, c, d, x[1], 0xa4beea44u, 4);
    CR_STEP(CR_H, d, a, b, c, x[4], 0x4bdecfa9u, 11);
    CR_STEP(CR_H, c, d, a, b, x[7], 0xf6bb4b60u, 16);
    CR_STEP(CR_H, b, c, d, a, x[10], 0xbebfbc70u, 23);
    CR_STEP(CR_H, a, b, c, d, x[13], 0x289b7ec6u, 4);
    CR_STEP(CR_H, d, a, b, c, x[0], 0xeaa127fau, 11);
    CR_STEP(CR_H, c, d, a, b, x[3], 0xd4ef3085u, 16);
    CR_STEP(CR_H, b, c, d, a, x[6], 0x04881d05u, 23);
    CR_STEP(CR_H, a, b, c, d, x[9], 0xd9d4d039u, 4);
    CR_STEP(CR_H, d, a, b, c, x[12], 0xe6db99e5u, 11);
    CR_STEP(CR_H, c, d, a, b, x[15], 0x1fa27cf8u, 16);
    CR_STEP(CR_H, b, c, d, a, x[2], 0xc4ac5665u, 23);
    // round 4: word k = 7j mod 16
    CR_STEP(CR_I, a, b, c, d, x[0], 0xf4292244u, 6);
    CR_STEP(CR_I, d, a, b, c, x[7], 0x432aff97u, 10);
    CR_STEP(CR_I, c, d, a, b, x[14], 0xab9423a7u, 15);
    CR_STEP(CR_I, b, c, d, a, x[5], 0xfc93a039u, 21);
    CR_STEP(CR_I, a, b, c, d, x[12], 0x655b59c3u, 6);
    CR_STEP(CR_I, d, a, b, c, x[3], 0x8f0ccc92u, 10);
    CR_STEP(CR_I, c, d, a, b, x[10], 0xffeff47du, 15);
    CR_STEP(CR_I, b, c, d, a, x[1], 0x85845dd1u, 21);
    CR_STEP(CR_I, a, b, c, d, x[8], 0x6fa87e4fu, 6);
    CR_STEP(CR_I, d, a, b, c, x[15], 0xfe2ce6e0u, 10);
    CR_STEP(CR_I, c, d, a, b, x[6], 0xa3014314u, 15);
    CR_STEP(CR_I, b, c, d, a, x[13], 0x4e0811a1u, 21);
    CR_STEP(CR_I, a, b, c, d, x[4], 0xf7537e82u, 6);
    CR_STEP(CR_I, d, a, b, c, x[11], 0xbd3af235u, 10);
    CR_STEP(CR_I, c, d, a, b, x[2], 0x2ad7d2bbu, 15);
    CR_STEP(CR_I, b, c, d, a, x[9], 0xeb86d391u, 21);
    st[0] += a;
    st[1] += b;
    st[2] += c;
    st[3] += d;
}

__device__ __forceinline__ void md5_init(uint32_t st[4])
{
    st[0] = 0x67452301u;
    st[1] = 0xefcdab89u;
    st[2] = 0x98badcfeu;
    st[3] = 0x10325476u;
}

// Final block(s): w[] holds the message's last r (< 64) bytes in its low words
// (any content beyond byte r); appends 0x80, zero fill and the 64-bit
// little-endian bit length, and compresses one or two blocks.
__device__ __forceinline__ void md5_finish(uint32_t st[4], const uint32_t w[16],
                                           uint32_t r, uint64_t total_len)
{
    uint32_t x[16];
#pragma unroll
    for (int k = 0; k < 16; k++) {
        int rem = (int)r - 4 * k;
        uint32_t keep = rem >= 4 ? 0xffffffffu : (rem > 0 ? ((1u << (8 * rem)) - 1u) : 0u);
        uint32_t pad = (rem >= 0 && rem < 4) ? (0x80u << (8 * rem)) : 0u;
        x[k] = (w[k] & keep) | pad;
    }
    const uint64_t bits = total_len << 3;
    if (r < 56) {
        x[14] = (uint32_t)bits;
        x[15] = (uint32_t)(bits >> 32);
        md5_compress(st, x);
    } else {
        md5_compress(st, x);
#pragma unroll
        for (int k = 0; k < 14; k++)
            x[k] = 0;
        x[14] = (uint32_t)bits;
        x[15] = (uint32_t)(bits >> 32);
        md5_compress(st, x);
    }
}

__device__ __forceinline__ void md5_unpack4(uint32_t x[16], const uint4 &v0,
                                            const uint4 &v1, const uint4 &v2,
                                            const uint4 &v3)
{
    x[0] = v0.x; x[1] = v0.y; x[2] = v0.z; x[3] = v0.w;
    x[4] = v1.x; x[5] = v1.y; x[6] = v1.z; x[7] = v1.w;
    x[8] = v2.x; x[9] = v2.y; x[10] = v2.z; x[11] = v2.w;
    x[12] = v3.x; x[13] = v3.y; x[14] = v3.z; x[15] = v3.w;
}

// MD5 of a message that starts on a 16-byte boundary.  Full blocks are read
// as 16-byte vectors, two blocks (128 B) per load group so each lane consumes
// whole 128-byte lines.
__device__ __forceinline__ void md5_message_a16(const uint8_t *__restrict__ p,
                                                uint64_t len, uint32_t st[4])
{
    md5_init(st);
    const uint4 *q = reinterpret_cast<const uint4 *>(p);
    const uint64_t nb = len >> 6;
    uint64_t b = 0;
    for (; b + 2 <= nb; b += 2) {
        const uint4 *r = q + 4 * b;
        uint4 v0 = r[0], v1 = r[1], v2 = r[2], v3 = r[3];
        uint4 v4 = r[4], v5 = r[5], v6 = r[6], v7 = r[7];
        uint32_t x[16];
        md5_unpack4(x, v0, v1, v2, v3);
        md5_compress(st, x);
        md5_unpack4(x, v4, v5, v6, v7);
        md5_compress(st, x);
    }
    if (b < nb) {
        const uint4 *r = q + 4 * b;
        uint4 v0 = r[0], v1 = r[1], v2 = r[2], v3 = r[3];
        uint32_t x[16];
        md5_unpack4(x, v0, v1, v2, v3);
        md5_compress(st, x);
    }
    // tail: r bytes at q + 4*nb, loaded only as far as they reach
    const uint32_t rb = (uint32_t)(len & 63);
    const uint4 *t = q + 4 * nb;
    uint4 z = make_uint4(0, 0, 0, 0);
    uint4 t0 = rb > 0 ? t[0] : z;
    uint4 t1 = rb > 16 ? t[1] : z;
    uint4 t2 = rb > 32 ? t[2] : z;
    uint4 t3 = rb > 48 ? t[3] : z;
    uint32_t w[16];
    md5_unpack4(w, t0, t1, t2, t3);
    md5_finish(st, w, rb, len);
}

// --- double-buffered loaders ---
//
// The message is consumed in chunks of D units.  Two register buffers
// alternate: the loads for the other buffer are issued before the current
// buffer is compressed, so each chunk's loads have a whole chunk of compute
// to arrive.  The loop body is [load B | compress A | load A' | compress B];
// the only wait that must be exact (before compressing B) sits inside one
// basic block, and the wait the compiler places at the loop header finds
// its loads already complete.  Look-ahead loads are unconditional, with the
// chunk index clamped to the last full chunk (always inside the message).

template <int D>
__device__ __forceinline__ void a16_load_chunk(uint4 (&r)[D][8], const uint4 *q, uint64_t c)
{
    const uint4 *b = q + (uint64_t)8 * D * c;
#pragma unroll
    for (int j = 0; j < D; j++)
#pragma unroll
        for (int k = 0; k < 8; k++)
            r[j][k] = b[8 * j + k];
}

template <int D>
__device__ __forceinline__ void a16_compress_chunk(uint32_t st[4], const uint4 (&r)[D][8])
{
#pragma unroll
    for (int j = 0; j < D; j++) {
        uint32_t x[16];
        md5_unpack4(x, r[j][0], r[j][1], r[j][2], r[j][3]);
        md5_compress(st, x);
        md5_unpack4(x, r[j][4], r[j][5], r[j][6], r[j][7]);
        md5_compress(st, x);
    }
}

// 16-byte-aligned message, chunks of D groups of 128 bytes.
template <int D>
__device__ __forceinline__ void md5_message_a16_db(const uint8_t *__restrict__ p,
                                                   uint64_t len, uint32_t st[4])
{
    md5_init(st);
    const uint4 *q = reinterpret_cast<const uint4 *>(p);
    const uint64_t nb = len >> 6;
    const uint64_t ng = nb >> 1;
    const uint64_t nc = ng / D;
    if (nc) {
        uint4 A[D][8], B[D][8];
        a16_load_chunk<D>(A, q, 0);
        uint64_t c = 0;
        for (; c + 1 < nc; c += 2) {
            // the barriers keep each chunk's loads ahead of the other
            // chunk's compression (the scheduler would sink them)
            a16_load_chunk<D>(B, q, c + 1);
            __builtin_amdgcn_sched_barrier(0);
            a16_compress_chunk<D>(st, A);
            __builtin_amdgcn_sched_barrier(0);
            a16_load_chunk<D>(A, q, c + 2 < nc ? c + 2 : nc - 1);
            __builtin_amdgcn_sched_barrier(0);
            a16_compress_chunk<D>(st, B);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (c < nc) // odd chunk count: A holds chunk nc - 1
            a16_compress_chunk<D>(st, A);
    }
    for (uint64_t g = nc * D; g < ng; ++g) {
        const uint4 *r = q + 8 * g;
        uint4 v0 = r[0], v1 = r[1], v2 = r[2], v3 = r[3];
        uint4 v4 = r[4], v5 = r[5], v6 = r[6], v7 = r[7];
        uint32_t x[16];
        md5_unpack4(x, v0, v1, v2, v3);
        md5_compress(st, x);
        md5_unpack4(x, v4, v5, v6, v7);
        md5_compress(st, x);
    }
    const uint4 z = make_uint4(0, 0, 0, 0);
    if (nb & 1) {
        const uint4 *r = q + 8 * ng;
        uint4 v0 = r[0], v1 = r[1], v2 = r[2], v3 = r[3];
        uint32_t x[16];
        md5_unpack4(x, v0, v1, v2, v3);
        md5_compress(st, x);
    }
    const uint32_t rb = (uint32_t)(len & 63);
    const uint4 *t = q + 4 * nb;
    uint4 t0 = rb > 0 ? t[0] : z;
    uint4 t1 = rb > 16 ? t[1] : z;
    uint4 t2 = rb > 32 ? t[2] : z;
    uint4 t3 = rb > 48 ? t[3] : z;
    uint32_t w[16];
    md5_unpack4(w, t0, t1, t2, t3);
    md5_finish(st, w, rb, len);
}

// MD5 of a message at any byte address.  Each block is read as 17 aligned
// dwords starting at the dword that holds its first byte (four 16-byte
// vectors with 4-byte alignment plus one dword) and realigned with
// v_alignbyte_b32 by the byte offset inside that dword.
__device__ __forceinline__ void md5_message_any(const uint8_t *__restrict__ p,
                                                uint64_t len, uint32_t st[4])
{
    md5_init(st);
    const uint32_t bs = (uint32_t)((uintptr_t)p & 3);
    const uint32_t *d = reinterpret_cast<const uint32_t *>(p - bs);
    const uint64_t nb = len >> 6;
    for (uint64_t b = 0; b < nb; ++b) {
        const uint32_t *r = d + 16 * b;
        u32x4a4 v0 = *reinterpret_cast<const u32x4a4 *>(r);
        u32x4a4 v1 = *reinterpret_cast<const u32x4a4 *>(r + 4);
        u32x4a4 v2 = *reinterpret_cast<const u32x4a4 *>(r + 8);
        u32x4a4 v3 = *reinterpret_cast<const u32x4a4 *>(r + 12);
        uint32_t e = bs ? r[16] : 0u;
        uint32_t u[17] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w,
                          v2.x, v2.y, v2.z, v2.w, v3.x, v3.y, v3.z, v3.w, e};
        uint32_t x[16];
#pragma unroll
        for (int k = 0; k < 16; k++)
            x[k] = __builtin_amdgcn_alignbyte(u[k + 1], u[k], bs);
        md5_compress(st, x);
    }
    // tail: rb bytes starting at byte offset bs of dword d[16*nb]; they span
    // at most ceil((bs + rb) / 4) dwords, and only those are read.
    const uint32_t rb = (uint32_t)(len & 63);
    const uint32_t *r = d + 16 * nb;
    const uint32_t span = rb ? (bs + rb + 3) >> 2 : 0u;
    uint32_t u[17];
#pragma unroll
    for (int k = 0; k < 17; k++)
        u[k] = (uint32_t)k < span ? r[k] : 0u;
    uint32_t w[16];
#pragma unroll
    for (int k = 0; k < 16; k++)
        w[k] = __builtin_amdgcn_alignbyte(u[k + 1], u[k], bs);
    md5_finish(st, w, rb, len);
}

// Any-alignment message (see md5_message_any), double-buffered in chunks of
// D blocks; each block slot holds the 17 dwords that cover it.  The extra
// dword of a block is read from an index clamped to the dword holding the
// message's last byte, so it stays readable even where it is not needed.
template <int D>
__device__ __forceinline__ void any_load_chunk(uint32_t (&r)[D][17], const uint32_t *d,
                                               uint64_t c, uint64_t dmax)
{
#pragma unroll
    for (int j = 0; j < D; j++) {
        const uint64_t bi = (uint64_t)D * c + j;
        const uint32_t *b = d + 16 * bi;
        u32x4a4 v0 = *reinterpret_cast<const u32x4a4 *>(b);
        u32x4a4 v1 = *reinterpret_cast<const u32x4a4 *>(b + 4);
        u32x4a4 v2 = *reinterpret_cast<const u32x4a4 *>(b + 8);
        u32x4a4 v3 = *reinterpret_cast<const u32x4a4 *>(b + 12);
        const uint64_t e16 = 16 * bi + 16 < dmax ? 16 * bi + 16 : dmax;
        r[j][0] = v0.x; r[j][1] = v0.y; r[j][2] = v0.z; r[j][3] = v0.w;
        r[j][4] = v1.x; r[j][5] = v1.y; r[j][6] = v1.z; r[j][7] = v1.w;
        r[j][8] = v2.x; r[j][9] = v2.y; r[j][10] = v2.z; r[j][11] = v2.w;
        r[j][12] = v3.x; r[j][13] = v3.y; r[j][14] = v3.z; r[j][15] = v3.w;
        r[j][16] = d[e16];
    }
}

template <int D>
__device__ __forceinline__ void any_compress_chunk(uint32_t st[4], const uint32_t (&r)[D][17],
                                                   uint32_t bs)
{
#pragma unroll
    for (int j = 0; j < D; j++) {
        uint32_t x[16];
#pragma unroll
        for (int k = 0; k < 16; k++)
            x[k] = __builtin_amdgcn_alignbyte(r[j][k + 1], r[j][k], bs);
        md5_compress(st, x);
    }
}

template <int D>
__device__ __forceinline__ void md5_message_any_db(const uint8_t *__restrict__ p,
                                                   uint64_t len, uint32_t st[4])
{
    md5_init(st);
    const uint32_t bs = (uint32_t)((uintptr_t)p & 3);
    const uint32_t *d = reinterpret_cast<const uint32_t *>(p - bs);
    const uint64_t nb = len >> 6;
    const uint64_t nc = nb / D;
    const uint64_t dmax = len ? (bs + len - 1) >> 2 : 0; // dword holding the last byte
    if (nc) {
        uint32_t A[D][17], B[D][17];
        any_load_chunk<D>(A, d, 0, dmax);
        uint64_t c = 0;
        for (; c + 1 < nc; c += 2) {
            any_load_chunk<D>(B, d, c + 1, dmax);
            __builtin_amdgcn_sched_barrier(0);
            any_compress_chunk<D>(st, A, bs);
            __builtin_amdgcn_sched_barrier(0);
            any_load_chunk<D>(A, d, c + 2 < nc ? c + 2 : nc - 1, dmax);
            __builtin_amdgcn_sched_barrier(0);
            any_compress_chunk<D>(st, B, bs);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (c < nc)
            any_compress_chunk<D>(st, A, bs);
    }
    for (uint64_t b = nc * D; b < nb; ++b) {
        uint32_t r1[1][17];
        const uint32_t *bb = d + 16 * b;
        u32x4a4 v0 = *reinterpret_cast<const u32x4a4 *>(bb);
        u32x4a4 v1 = *reinterpret_cast<const u32x4a4 *>(bb + 4);
        u32x4a4 v2 = *reinterpret_cast<const u32x4a4 *>(bb + 8);
        u32x4a4 v3 = *reinterpret_cast<const u32x4a4 *>(bb + 12);
        const uint64_t e16 = 16 * b + 16 < dmax ? 16 * b + 16 : dmax;
        r1[0][0] = v0.x; r1[0][1] = v0.y; r1[0][2] = v0.z; r1[0][3] = v0.w;
        r1[0][4] = v1.x; r1[0][5] = v1.y; r1[0][6] = v1.z; r1[0][7] = v1.w;
        r1[0][8] = v2.x; r1[0][9] = v2.y; r1[0][10] = v2.z; r1[0][11] = v2.w;
        r1[0][12] = v3.x; r1[0][13] = v3.y; r1[0][14] = v3.z; r1[0][15] = v3.w;
        r1[0][16] = d[e16];
        any_compress_chunk<1>(st, r1, bs);
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
    md5_finish(st, w, rb, len);
}

__device__ __forceinline__ void md5_store(uint8_t *__restrict__ out, const uint32_t st[4])
{
    *reinterpret_cast<uint4 *>(out) = make_uint4(st[0], st[1], st[2], st[3]);
}

} // namespace crystal
