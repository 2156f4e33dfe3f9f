// Content-defined chunking kernels.
//
// 1. Candidates.  Lane L owns bytes [4096 L, 4096 L + 4096) and rolls the
//    48-byte window hash W_i = W_{i-1} B - in[i-48] B^48 + in[i] across them,
//    after a 48-byte warm-up over the bytes just before its range.  A
//    candidate is (W_i & mask) == 0.  Only W mod 2^k with 2^k >= mask
//    matters (reduction mod 2^k is a ring homomorphism of Z/2^64), so masks
//    of up to 32 bits roll in 32-bit registers and still decide exactly the
//    same positions; wider masks roll in 64 bits.
//    Output is a two-level bitmap: level 1 holds one bit per byte, stored
//    only for nonzero 64-bit words; level 2 holds, per range, a 64-bit mask
//    of which level-1 words are nonzero.  Plus a per-range candidate count.
//
// 2. Selection (the chunk rule is a sequential chain: each chunk start fixes
//    the next).  The input is split into tiles of P >= max_len bytes.  Each
//    tile walks the chain speculatively from D bytes before its tile (D = 2P;
//    inputs of up to 256 tiles use about two mean chunk lengths, at least
//    16 KiB), records the starts that fall inside its tile and the first
//    start past it (its exit).  Two chains that reach the same start agree
//    from then on, so if the exit of tile t-1 equals the first start tile t
//    recorded, tile t's starts are exact; tile 0 starts at 0 and is exact.
//    Verification checks every tile; tiles that fail are re-walked from the
//    true entry by a repair pass (rare on real data).  A scan of per-tile
//    counts then packs the starts into the ends array.  Inputs of up to 1024
//    tiles do all of this after the walk, and the chunk order, in one
//    workgroup; larger ones verify, repair and scan in one workgroup and
//    pack (counting the chunks' length classes for the order) in parallel.
#include "internal.h"

namespace crystal {

// ------------------------------------------------------------ candidates

// Byte t (0..15) of a 16-byte vector.
__device__ __forceinline__ uint32_t vbyte(const uint4 &v, int t)
{
    const uint32_t w = (t < 4) ? v.x : (t < 8) ? v.y : (t < 12) ? v.z : v.w;
    return (w >> (8 * (t & 3))) & 0xffu;
}

__device__ __forceinline__ uint4 load_vec(const uint8_t *__restrict__ in, uint64_t pos,
                                          uint64_t n)
{
    // pos is 16-byte aligned; a vector is read only if it holds an input byte.
    if (pos < n)
        return *reinterpret_cast<const uint4 *>(in + pos);
    return make_uint4(0, 0, 0, 0);
}

// Roll 16 positions: `cin` holds the entering bytes, `cout` the bytes that
// leave (48 positions earlier).  Returns the 16-bit candidate mask.
template <typename WT>
__device__ __forceinline__ uint32_t roll16(WT &w, const uint4 &cin, const uint4 &cout,
                                          WT B, WT B48, WT M)
{
    uint32_t bits = 0;
#pragma unroll
    for (int t = 0; t < 16; t++) {
        w = w * B + (WT)vbyte(cin, t) - (WT)vbyte(cout, t) * B48;
        bits |= ((w & M) == 0 ? 1u : 0u) << t;
    }
    return bits;
}

template <typename WT>
__device__ __forceinline__ void roll16_store(WT &w, const uint4 &cin, const uint4 &cout,
                                             WT B, WT B48, uint64_t *__restrict__ dst,
                                             uint64_t pos, uint64_t n)
{
#pragma unroll
    for (int t = 0; t < 16; t++) {
        w = w * B + (WT)vbyte(cin, t) - (WT)vbyte(cout, t) * B48;
        const uint64_t i = pos + t;
        if (i < n)
            dst[i] = (i + 1 >= kWindow) ? (uint64_t)w : 0;
    }
}

// ------------------------------------------ two parts per lane, 16-bit halves
// A mask of at most 15 bits reads only W mod 2^16, and W mod 2^16 rolls
// exactly in 16-bit arithmetic (reduction mod 2^16 is a ring homomorphism).
// So each lane rolls two parts at once, one in each 16-bit half of a
// register, with packed multiply-adds (v_pk_mad_u16): about 4.5 VALU
// instructions per byte against about 9 for the 32-bit roll, and no 32-bit
// multiplies.  The candidate test needs no compare either: for M < 2^15,
// (W & M) - 1 taken in 16 bits has its top bit set exactly when W & M == 0.
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t vword(const uint4 &v, int t)
{
    return (t < 4) ? v.x : (t < 8) ? v.y : (t < 12) ? v.z : v.w;
}

// Byte t of a in the low half, byte t of b in the high half.  The permute
// selector picks from the 8 bytes {b word (4..7), a word (0..3)}; 0x0c
// yields a zero byte.
__device__ __forceinline__ u16x2 pair_bytes(const uint4 &a, const uint4 &b, int t)
{
    const uint32_t sel = 0x0c000c00u | ((4u + (uint32_t)(t & 3)) << 16) | (uint32_t)(t & 3);
    return __builtin_bit_cast(u16x2, __builtin_amdgcn_perm(vword(b, t), vword(a, t), sel));
}

// Roll 16 positions of both parts.  Bit t of the result flags part A's
// position t, bit 16 + t part B's: each step shifts the flags right by one
// and adds the new ones at bits 15 and 31, so that after 16 steps step t's
// flags sit at t and 16 + t without crossing between the halves.
__device__ __forceinline__ uint32_t roll16x2(u16x2 &w, const uint4 &ia, const uint4 &ib,
                                             const uint4 &oa, const uint4 &ob, u16x2 B,
                                             u16x2 nB48, uint32_t M2)
{
    const u16x2 one = {1, 1};
    uint32_t bits = 0;
#pragma unroll
    for (int t = 0; t < 16; t++) {
        w = w * B + pair_bytes(ia, ib, t);
        w = pair_bytes(oa, ob, t) * nB48 + w; // - out * B^48
        const u16x2 z = __builtin_bit_cast(u16x2, __builtin_bit_cast(uint32_t, w) & M2);
        const uint32_t f = __builtin_bit_cast(uint32_t, (u16x2)(z - one));
        bits = (bits >> 1) | (f & 0x80008000u);
    }
    return bits;
}

// Candidate bitmap for masks of at most 15 bits.  2^lgk consecutive lanes
// share a 4 KiB range; lane `sub` rolls its parts 2 sub and 2 sub + 1 of
// 4096 >> (lgk + 1) bytes, each after its own 48-byte warm-up, so the launch
// shape and the bytes per lane are those of k_cdc_roll.
__global__ __launch_bounds__(256) void k_cdc_roll_x2(const uint8_t *__restrict__ in, uint64_t n,
                                                     uint32_t b16, uint32_t nb48_16, uint32_t M2,
                                                     uint64_t *__restrict__ l1,
                                                     uint64_t *__restrict__ l2,
                                                     uint32_t *__restrict__ cnt, uint32_t lgk)
{
    const uint64_t lane = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t L = lane >> lgk;
    const uint32_t sub = (uint32_t)(lane & ((1u << lgk) - 1));
    const uint64_t part = kRangeBytes >> (lgk + 1); // a multiple of 64 bytes, >= 128
    if (L * kRangeBytes >= n)
        return; // the range's lanes all leave here together
    const uint64_t a0 = L * kRangeBytes + 2ull * sub * part, b0 = a0 + part;
    const uint64_t a1 = a0 >= n ? a0 : ((a0 + part < n) ? a0 + part : n);
    const uint64_t b1 = b0 >= n ? b0 : ((b0 + part < n) ? b0 + part : n);
    const uint32_t ga = (uint32_t)(2ull * sub * (part >> 6)); // first level-1 word of part A
    const uint32_t gb = ga + (uint32_t)(part >> 6);
    const u16x2 B = __builtin_bit_cast(u16x2, b16 | (b16 << 16));
    const u16x2 nB48 = __builtin_bit_cast(u16x2, nb48_16 | (nb48_16 << 16));
    const uint4 zero = make_uint4(0, 0, 0, 0);

    // Warm-up over the 48 bytes before each part (part A of the input's
    // first lane has none: its half stays 0, as after rolling in zeros).
    u16x2 w = {0, 0};
    uint4 pa1 = zero, pa2 = zero, pa3 = zero;
    if (a0 >= 48) {
        pa1 = load_vec(in, a0 - 48, n);
        pa2 = load_vec(in, a0 - 32, n);
        pa3 = load_vec(in, a0 - 16, n);
    }
    uint4 pb1 = load_vec(in, b0 - 48, n), pb2 = load_vec(in, b0 - 32, n),
          pb3 = load_vec(in, b0 - 16, n);
    roll16x2(w, pa1, pb1, zero, zero, B, nB48, M2);
    roll16x2(w, pa2, pb2, zero, zero, B, nB48, M2);
    roll16x2(w, pa3, pb3, zero, zero, B, nB48, M2);

    // 128 bytes of each part per step, loaded together, so that each
    // 128-byte line is requested once and used at once (taking a line in
    // two 64-byte halves a step apart let the cache evict it in between and
    // fetch it twice: 1.36x the input)
    uint64_t l2bits = 0;
    uint32_t count = 0;
    const uint32_t nsteps = (uint32_t)((a1 - a0 + 127) >> 7); // part B is never longer
    uint4 ca[8], cb[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
        ca[k] = load_vec(in, a0 + 16 * k, n);
        cb[k] = load_vec(in, b0 + 16 * k, n);
    }
    for (uint32_t g = 0; g < nsteps; g++) {
        const uint64_t pa = a0 + 128ull * g, pb = b0 + 128ull * g;
        uint4 na[8], nb[8];
#pragma unroll
        for (int k = 0; k < 8; k++)
            na[k] = nb[k] = zero;
        if (g + 1 < nsteps) {
#pragma unroll
            for (int k = 0; k < 8; k++) {
                na[k] = load_vec(in, pa + 128 + 16 * k, n);
                nb[k] = load_vec(in, pb + 128 + 16 * k, n);
            }
        }
        // leaving bytes of vector q are those of the vector 48 bytes back
        uint32_t r[8];
        r[0] = roll16x2(w, ca[0], cb[0], pa1, pb1, B, nB48, M2);
        r[1] = roll16x2(w, ca[1], cb[1], pa2, pb2, B, nB48, M2);
        r[2] = roll16x2(w, ca[2], cb[2], pa3, pb3, B, nB48, M2);
#pragma unroll
        for (int q = 3; q < 8; q++)
            r[q] = roll16x2(w, ca[q], cb[q], ca[q - 3], cb[q - 3], B, nB48, M2);
#pragma unroll
        for (int h = 0; h < 2; h++) {
            uint64_t wa = (uint64_t)((r[4 * h] & 0xffffu) | (r[4 * h + 1] << 16)) |
                          ((uint64_t)((r[4 * h + 2] & 0xffffu) | (r[4 * h + 3] << 16)) << 32);
            uint64_t wb = (uint64_t)((r[4 * h] >> 16) | (r[4 * h + 1] & 0xffff0000u)) |
                          ((uint64_t)((r[4 * h + 2] >> 16) | (r[4 * h + 3] & 0xffff0000u)) << 32);
            const uint64_t qa = pa + 64 * h, qb = pb + 64 * h;
            // positions below 47 have no full window; positions past a
            // part's end are outside it (part B may end first, or be empty)
            if (qa < 47)
                wa &= ~0ull << (47 - qa);
            if (qa >= a1)
                wa = 0;
            else if (qa + 64 > a1)
                wa &= (1ull << (a1 - qa)) - 1;
            if (qb >= b1)
                wb = 0;
            else if (qb + 64 > b1)
                wb &= (1ull << (b1 - qb)) - 1;
            if (wa) {
                l1[qa >> 6] = wa;
                l2bits |= 1ull << (ga + 2 * g + h);
                count += __popcll(wa);
            }
            if (wb) {
                l1[qb >> 6] = wb;
                l2bits |= 1ull << (gb + 2 * g + h);
                count += __popcll(wb);
            }
        }
        pa1 = ca[5];
        pa2 = ca[6];
        pa3 = ca[7];
        pb1 = cb[5];
        pb2 = cb[6];
        pb3 = cb[7];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            ca[k] = na[k];
            cb[k] = nb[k];
        }
    }
    for (uint32_t o = 1; o < (1u << lgk); o <<= 1) {
        l2bits |= __shfl_xor(l2bits, (int)o);
        count += __shfl_xor(count, (int)o);
    }
    if (sub == 0) {
        l2[L] = l2bits;
        cnt[L] = count;
    }
}

// MODE 0: candidate bitmap.  MODE 1: dump the 64-bit window hash per byte.
//
// 2^lgk consecutive lanes share one 4 KiB range: each rolls its own
// (4096 >> lgk)-byte part after its own warm-up, and the lanes combine the
// range's level-2 mask and count with shuffles.  A small input thus fills
// more of the chip (one lane per range would leave each lane a long serial
// roll); large inputs use one lane per range.
template <typename WT, int MODE>
__global__ __launch_bounds__(256) void k_cdc_roll(const uint8_t *__restrict__ in,
                                                  uint64_t n, uint64_t base, uint64_t b48,
                                                  uint64_t mask, uint64_t *__restrict__ l1,
                                                  uint64_t *__restrict__ l2,
                                                  uint32_t *__restrict__ cnt,
                                                  uint64_t *__restrict__ wout, uint32_t lgk)
{
    const uint64_t lane = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t L = lane >> lgk;                        // range
    const uint32_t sub = (uint32_t)(lane & ((1u << lgk) - 1)); // part of the range
    const uint64_t part = kRangeBytes >> lgk;              // a multiple of 64 bytes
    if (L * kRangeBytes >= n)
        return; // the range's lanes all leave here together
    const uint64_t r0 = L * kRangeBytes + sub * part;
    const uint64_t r1 = r0 >= n ? r0 : ((r0 + part < n) ? r0 + part : n);
    const uint32_t g_base = (uint32_t)(sub * (part >> 6)); // first level-1 word of the part
    const WT B = (WT)base, B48 = (WT)b48, M = (WT)mask;
    const uint4 zero = make_uint4(0, 0, 0, 0);

    // Warm-up: the 48 bytes before r0 enter with nothing leaving, which
    // leaves W equal to the window hash ending at r0 - 1.
    WT w = 0;
    uint4 p1 = zero, p2 = zero, p3 = zero;
    if (r0 >= 48) {
        p1 = load_vec(in, r0 - 48, n);
        p2 = load_vec(in, r0 - 32, n);
        p3 = load_vec(in, r0 - 16, n);
        roll16<WT>(w, p1, zero, B, 0, M);
        roll16<WT>(w, p2, zero, B, 0, M);
        roll16<WT>(w, p3, zero, B, 0, M);
    }

    uint64_t l2bits = 0;
    uint32_t count = 0;
    const uint32_t ngroups = (uint32_t)((r1 - r0 + 63) >> 6);
    uint4 c0 = load_vec(in, r0, n), c1 = load_vec(in, r0 + 16, n);
    uint4 c2 = load_vec(in, r0 + 32, n), c3 = load_vec(in, r0 + 48, n);
    for (uint32_t g = 0; g < ngroups; g++) {
        const uint64_t pos = r0 + 64ull * g;
        // prefetch the next 64 bytes while this group is rolled
        uint4 n0 = zero, n1 = zero, n2 = zero, n3 = zero;
        if (g + 1 < ngroups) {
            n0 = load_vec(in, pos + 64, n);
            n1 = load_vec(in, pos + 80, n);
            n2 = load_vec(in, pos + 96, n);
            n3 = load_vec(in, pos + 112, n);
        }
        if (MODE == 0) {
            // leaving bytes of vector q are those of the vector 48 bytes back
            uint64_t word = (uint64_t)roll16<WT>(w, c0, p1, B, B48, M);
            word |= (uint64_t)roll16<WT>(w, c1, p2, B, B48, M) << 16;
            word |= (uint64_t)roll16<WT>(w, c2, p3, B, B48, M) << 32;
            word |= (uint64_t)roll16<WT>(w, c3, c0, B, B48, M) << 48;
            // positions below 47 have no full window; positions >= r1 are
            // outside the range
            if (pos < 47)
                word &= ~0ull << (47 - pos);
            if (pos + 64 > r1)
                word &= (r1 - pos >= 64) ? ~0ull : ((1ull << (r1 - pos)) - 1);
            if (word) {
                l1[pos >> 6] = word;
                l2bits |= 1ull << (g_base + g);
                count += __popcll(word);
            }
        } else {
            roll16_store<WT>(w, c0, p1, B, B48, wout, pos, r1);
            roll16_store<WT>(w, c1, p2, B, B48, wout, pos + 16, r1);
            roll16_store<WT>(w, c2, p3, B, B48, wout, pos + 32, r1);
            roll16_store<WT>(w, c3, c0, B, B48, wout, pos + 48, r1);
        }
        p1 = c1;
        p2 = c2;
        p3 = c3;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    if (MODE == 0) {
        // the lanes of one range are consecutive within a wave
        for (uint32_t o = 1; o < (1u << lgk); o <<= 1) {
            l2bits |= __shfl_xor(l2bits, (int)o);
            count += __shfl_xor(count, (int)o);
        }
        if (sub == 0) {
            l2[L] = l2bits;
            cnt[L] = count;
        }
    }
}

// Lanes per range (log2) for an input of n_ranges ranges: the most, up to
// 16, that keep the launch within about one wave per SIMD (256 CUs x 4
// SIMDs x 64 lanes), beyond which smaller parts only add warm-ups.
static uint32_t roll_lanes_log2(uint64_t n_ranges)
{
    const uint64_t target = 256 * 4 * 64;
    uint32_t lg = 0;
    while (lg < 4 && (n_ranges << (lg + 1)) <= target)
        lg++;
    return lg;
}

// ------------------------------------------------------------------ scans
// Exclusive scan of n u32 counts into u64 offsets by one workgroup of 1024
// threads; *total receives the sum.  Adequate for the per-range and
// per-tile count arrays (<= a few hundred thousand entries).
__global__ __launch_bounds__(1024) void k_scan_u32(const uint32_t *__restrict__ in,
                                                   uint64_t n, uint64_t *__restrict__ out,
                                                   uint64_t *__restrict__ total)
{
    __shared__ uint64_t wsum[16];
    __shared__ uint64_t carry_s;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0)
        carry_s = 0;
    __syncthreads();
    for (uint64_t base = 0; base < n; base += 1024) {
        const uint64_t i = base + tid;
        const uint64_t v = i < n ? in[i] : 0;
        // inclusive wave scan
        uint64_t x = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            uint64_t y = __shfl_up(x, d, 64);
            if (lane >= (uint32_t)d)
                x += y;
        }
        if (lane == 63)
            wsum[wv] = x;
        __syncthreads();
        uint64_t before = carry_s;
        for (uint32_t k = 0; k < wv; k++)
            before += wsum[k];
        if (i < n)
            out[i] = before + x - v;
        __syncthreads();
        if (tid == 1023)
            carry_s = before + x;
        __syncthreads();
    }
    if (tid == 0)
        *total = carry_s;
}

// Candidate list from the bitmap: range L writes its positions at its scanned
// offset.  Positions beyond cap are dropped (the count is still exact).
__global__ __launch_bounds__(256) void k_cdc_compact(const uint64_t *__restrict__ l1,
                                                     const uint64_t *__restrict__ l2,
                                                     const uint64_t *__restrict__ rscan,
                                                     uint64_t n_ranges,
                                                     uint64_t *__restrict__ cand,
                                                     uint64_t cap)
{
    const uint64_t L = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (L >= n_ranges)
        return;
    uint64_t o = rscan[L];
    uint64_t m = l2[L];
    while (m) {
        const uint32_t g = __builtin_ctzll(m);
        m &= m - 1;
        uint64_t bits = l1[L * 64 + g];
        while (bits) {
            const uint32_t b = __builtin_ctzll(bits);
            bits &= bits - 1;
            if (o < cap)
                cand[o] = L * kRangeBytes + 64ull * g + b;
            o++;
        }
    }
}

// Chunk length classes of the longest-first chunk order (see "chunk order"
// below); the selection's packing kernel counts them too.
constexpr uint32_t kLenClasses = 64;

// Class 0 holds the longest chunks (>= 63 KiB + 1 byte, also every longer
// chunk when max_len exceeds 64 KiB), class 63 the shortest (<= 1 KiB).
__device__ __forceinline__ uint32_t len_class(uint64_t len)
{
    const uint64_t c = len ? (len - 1) >> 10 : 0;
    return kLenClasses - 1 - (uint32_t)(c < kLenClasses - 1 ? c : kLenClasses - 1);
}

__device__ __forceinline__ uint64_t chunk_len(const uint64_t *ends, uint64_t k)
{
    return ends[k] - (k ? ends[k - 1] : 0);
}

// -------------------------------------------------------------- selection

struct SelArgs {
    const uint64_t *l1, *l2;
    uint64_t n, min_len, max_len, tile_bytes, warm_bytes;
    uint32_t n_tiles, tile_cap;
    uint64_t *exit_, *first;
    uint32_t *tcnt;
    uint64_t *starts;
    uint32_t *flags;
    uint32_t *bad; // [0] = count of tiles failing verification, [1] = overflow
};

constexpr uint64_t kNone = ~0ull;

// First candidate position c with lo <= c <= hi, or kNone.
__device__ __forceinline__ uint64_t first_cand(const SelArgs &a, uint64_t lo, uint64_t hi)
{
    if (lo > hi)
        return kNone;
    const uint64_t wlo = lo >> 6, whi = hi >> 6;
    uint64_t w = wlo;
    while (w <= whi) {
        const uint64_t R = w >> 6;
        const uint64_t m = a.l2[R] & (~0ull << (w & 63));
        if (m == 0) {
            w = (R + 1) << 6;
            continue;
        }
        const uint64_t g = (R << 6) + __builtin_ctzll(m);
        if (g > whi)
            return kNone;
        uint64_t bits = a.l1[g];
        if (g == wlo)
            bits &= ~0ull << (lo & 63);
        if (bits) {
            const uint64_t c = (g << 6) + __builtin_ctzll(bits);
            return c <= hi ? c : kNone;
        }
        w = g + 1;
    }
    return kNone;
}

// Start of the chunk after the one starting at s (< n): the first candidate
// i with i+1-s >= min_len, unless the length reaches max_len first; the
// input end if neither happens.
__device__ __forceinline__ uint64_t next_start(const SelArgs &a, uint64_t s)
{
    const uint64_t lo = s + a.min_len - 1;
    uint64_t hi = s + a.max_len - 1;
    if (hi > a.n - 1)
        hi = a.n - 1;
    const uint64_t c = first_cand(a, lo, hi);
    if (c != kNone)
        return c + 1;
    if (s + a.max_len <= a.n)
        return s + a.max_len;
    return a.n;
}

// Walk from `s` recording the starts inside tile t; returns the exit.
__device__ uint64_t walk_tile(const SelArgs &a, uint32_t t, uint64_t s)
{
    const uint64_t lt = (uint64_t)t * a.tile_bytes;
    uint64_t lt1 = lt + a.tile_bytes;
    if (lt1 > a.n)
        lt1 = a.n;
    uint32_t c = 0;
    uint64_t first = kNone;
    uint64_t *dst = a.starts + (uint64_t)t * a.tile_cap;
    while (s < lt1) {
        if (s >= lt) {
            if (c < a.tile_cap)
                dst[c] = s;
            else
                a.bad[1] = 1; // cannot happen when tile_cap >= ceil(P/min)
            if (c == 0)
                first = s;
            c++;
        }
        s = next_start(a, s);
    }
    a.first[t] = (c ? first : s);
    a.tcnt[t] = c;
    a.exit_[t] = s;
    return s;
}

// Inclusive scan of x over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t x, uint32_t lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= (uint32_t)d)
            x += y;
    }
    return x;
}

// Candidates (and level-1 words holding them) one tile's span may keep in LDS.
constexpr uint32_t kSelCap = 2048;

// One wave per tile.  A lone lane walking the chain through the bitmaps pays
// two or three dependent global loads per chunk.  Instead the wave first
// gathers, in LDS and in position order, every candidate the walk can look
// at: the span from its speculative start s0 to the last position its final
// step can reach (tile end - 1 + max_len).  Lanes read the span's level-2
// words in parallel, list the set bits (the nonzero level-1 words), read
// those in parallel and expand them into positions, relative to the span's
// first range.  Lane 0 then walks the chain in LDS, keeping a cursor into
// the sorted list (chunk starts only increase, so it never moves back).  A
// span with more than kSelCap candidates, or wider than 4 GiB, is walked
// through global memory as before.
__global__ __launch_bounds__(64) void k_sel_walk(SelArgs a)
{
    __shared__ uint32_t words[kSelCap]; // level-1 word index - R0 * 64
    __shared__ uint32_t cand[kSelCap];  // candidate position - R0 * 4096
    const uint32_t t = blockIdx.x;
    const uint32_t lane = threadIdx.x;
    if (t >= a.n_tiles)
        return;
    const uint64_t lt = (uint64_t)t * a.tile_bytes;
    const uint64_t lt1 = a.n - lt < a.tile_bytes ? a.n : lt + a.tile_bytes;
    const uint64_t s0 = lt > a.warm_bytes ? lt - a.warm_bytes : 0;
    const uint64_t e = a.n - lt1 < a.max_len ? a.n : lt1 + a.max_len;
    const uint64_t R0 = s0 / kRangeBytes, R1 = (e - 1) / kRangeBytes;
    const uint64_t base = R0 * kRangeBytes;
    bool fits = (R1 + 1 - R0) * kRangeBytes <= (1ull << 32);
    uint32_t nw = 0, nc = 0;
    for (uint64_t Rb = R0; fits && Rb <= R1; Rb += 64) {
        const uint64_t R = Rb + lane;
        uint64_t m = R <= R1 ? a.l2[R] : 0;
        const uint32_t k = (uint32_t)__popcll(m);
        const uint32_t x = wave_scan_incl(k, lane);
        const uint32_t tot = __shfl(x, 63, 64);
        if (nw + tot > kSelCap) {
            fits = false;
            break;
        }
        uint32_t o = nw + x - k;
        const uint32_t w0 = (uint32_t)((R - R0) << 6);
        while (m) {
            words[o++] = w0 + (uint32_t)__builtin_ctzll(m);
            m &= m - 1;
        }
        nw += tot;
    }
    __syncthreads();
    for (uint32_t wb = 0; fits && wb < nw; wb += 64) {
        const uint32_t i = wb + lane;
        uint32_t wi = 0;
        uint64_t bits = 0;
        if (i < nw) {
            wi = words[i];
            bits = a.l1[(R0 << 6) + wi];
        }
        const uint32_t k = (uint32_t)__popcll(bits);
        const uint32_t x = wave_scan_incl(k, lane);
        const uint32_t tot = __shfl(x, 63, 64);
        if (nc + tot > kSelCap) {
            fits = false;
            break;
        }
        uint32_t o = nc + x - k;
        while (bits) {
            cand[o++] = (wi << 6) + (uint32_t)__builtin_ctzll(bits);
            bits &= bits - 1;
        }
        nc += tot;
    }
    __syncthreads();
    if (lane != 0)
        return;
    if (!fits) {
        walk_tile(a, t, s0);
        return;
    }
    uint32_t c = 0, p = 0;
    uint64_t first = kNone, s = s0;
    uint64_t *dst = a.starts + (uint64_t)t * a.tile_cap;
    while (s < lt1) {
        if (s >= lt) {
            if (c < a.tile_cap)
                dst[c] = s;
            else
                a.bad[1] = 1;
            if (c == 0)
                first = s;
            c++;
        }
        // the chunk's end: first candidate in [s + min - 1, min(s + max - 1, n - 1)]
        const uint64_t lo = s + a.min_len - 1;
        uint64_t hi = s + a.max_len - 1;
        if (hi > a.n - 1)
            hi = a.n - 1;
        while (p < nc && base + cand[p] < lo)
            p++;
        if (p < nc && base + cand[p] <= hi)
            s = base + cand[p] + 1;
        else
            s = s + a.max_len <= a.n ? s + a.max_len : a.n;
    }
    a.first[t] = (c ? first : s);
    a.tcnt[t] = c;
    a.exit_[t] = s;
}

// Copy tile t's c starts to ends[o - 1 ...] (start number j >= 1 is end j-1;
// entries past cap are dropped).  Eight loads are issued before their
// stores, so a tile costs one or two memory round trips instead of c.
__device__ __forceinline__ void emit_tile(const SelArgs &a, uint32_t t, uint32_t c, uint64_t o,
                                          uint64_t *__restrict__ ends, uint64_t cap)
{
    const uint64_t *src = a.starts + (uint64_t)t * a.tile_cap;
    if (c > a.tile_cap)
        c = a.tile_cap; // cannot happen: starts in a tile lie min_len apart
    for (uint32_t i = 0; i < c; i += 8) {
        uint64_t v[8];
#pragma unroll
        for (uint32_t q = 0; q < 8; q++)
            v[q] = i + q < c ? src[i + q] : 0;
#pragma unroll
        for (uint32_t q = 0; q < 8; q++) {
            const uint64_t k = o + i + q;
            if (i + q < c && k >= 1 && k - 1 < cap)
                ends[k - 1] = v[q];
        }
    }
}

// Pack tile t's starts into the ends array (start k >= 1 is end k-1; the
// last end is n).  With `hist` given, also count the chunks (below hcap) per
// length class, which the longest-first order needs: the chunk at a tile's
// last start ends at the tile's exit, the true next start once verification
// and repair are done.  A repair re-walks, in order, every tile whose entry
// disagrees with the true chain, so a repaired exit that moved is checked
// against the next tile in turn.
__global__ __launch_bounds__(64) void k_sel_emit(SelArgs a, const uint64_t *__restrict__ toff,
                                                 const uint64_t *__restrict__ total,
                                                 uint64_t *__restrict__ n_chunks,
                                                 uint64_t *__restrict__ ends, uint64_t cap,
                                                 uint32_t *__restrict__ hist, uint64_t hcap)
{
    __shared__ uint32_t h[kLenClasses]; // one entry per lane of the 64-lane group
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (hist) {
        h[threadIdx.x] = 0;
        __syncthreads();
    }
    if (t < a.n_tiles) {
        const uint32_t c = a.tcnt[t];
        const uint64_t o = toff[t];
        emit_tile(a, t, c, o, ends, cap);
        if (hist) {
            const uint64_t *src = a.starts + (uint64_t)t * a.tile_cap;
            const uint32_t cc = c < a.tile_cap ? c : a.tile_cap;
            for (uint32_t i = 0; i < cc && o + i < hcap; i++) {
                const uint64_t nx = i + 1 < cc ? src[i + 1] : a.exit_[t];
                atomicAdd(&h[len_class(nx - src[i])], 1u);
            }
        }
        if (t == a.n_tiles - 1) {
            const uint64_t m = *total; // number of chunk starts = number of chunks
            if (m >= 1 && m - 1 < cap)
                ends[m - 1] = a.n;
            *n_chunks = m;
        }
    }
    if (hist) {
        __syncthreads();
        if (h[threadIdx.x])
            atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
    }
}

// Past one finishing workgroup's tiles: verification, the serial repair and
// the scan of the tiles' counts in one workgroup (and the zeroing of the
// length-class counts k_sel_emit adds to), in place of four launches.
// Verification reads the tiles strided (coalesced); the scan gives thread i
// the tiles [i T, (i + 1) T).
__global__ __launch_bounds__(1024) void k_sel_verify_scan(SelArgs a, uint64_t *__restrict__ toff,
                                                          uint64_t *__restrict__ total,
                                                          uint32_t *__restrict__ hist)
{
    __shared__ uint32_t s_bad;
    __shared__ uint64_t wsum[16];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0)
        s_bad = 0;
    if (hist && tid < kLenClasses)
        hist[tid] = 0;
    __syncthreads();
    uint32_t bad = 0;
    for (uint32_t u = tid; u < a.n_tiles; u += 1024)
        bad += u >= 1 && a.exit_[u - 1] != a.first[u];
    if (bad)
        atomicAdd(&s_bad, bad);
    __syncthreads();
    if (s_bad) {
        if (tid == 0) {
            for (uint32_t u = 1; u < a.n_tiles; u++) {
                const uint64_t entry = a.exit_[u - 1];
                if (entry != a.first[u])
                    walk_tile(a, u, entry);
            }
        }
        __syncthreads();
    }
    const uint32_t T = (a.n_tiles + 1023) / 1024;
    const uint32_t u0 = tid * T < a.n_tiles ? tid * T : a.n_tiles;
    const uint32_t u1 = u0 + T < a.n_tiles ? u0 + T : a.n_tiles;
    uint64_t c = 0;
    for (uint32_t u = u0; u < u1; u++)
        c += a.tcnt[u];
    uint64_t x = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t y = __shfl_up(x, d, 64);
        if (lane >= (uint32_t)d)
            x += y;
    }
    if (lane == 63)
        wsum[wv] = x;
    __syncthreads();
    uint64_t before = 0, tot = 0;
    for (uint32_t k = 0; k < 16; k++) {
        before += k < wv ? wsum[k] : 0;
        tot += wsum[k];
    }
    uint64_t o = before + x - c;
    for (uint32_t u = u0; u < u1; u++) {
        toff[u] = o;
        o += a.tcnt[u];
    }
    if (tid == 0)
        *total = tot;
}

__global__ void k_store_zero_u64(uint64_t *p)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *p = 0;
}

// ---------------------------------------------------------------- launchers

// ------------------------------------------------------------ chunk order
// The chunk digests are one serial MD5 chain per chunk, and a wave runs as
// long as its longest lane.  Handing chunks to lanes longest first (in 1 KiB
// length classes) gives each wave 64 chains of nearly equal length and
// starts the longest chains first: for 256 MiB of random input (26 K chunks,
// the longest 1025 compressions) that measured 0.66 ms against 1.0 ms in
// index order.  Counting sort: class histogram, scan, scatter.


// One chunk per lane; per-workgroup class counts in LDS, added to hist.
__global__ __launch_bounds__(256) void k_chunk_hist(const uint64_t *__restrict__ ends,
                                                    const uint64_t *__restrict__ n_chunks,
                                                    uint64_t cap, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[kLenClasses];
    if (threadIdx.x < kLenClasses)
        h[threadIdx.x] = 0;
    __syncthreads();
    uint64_t nc = *n_chunks;
    nc = nc < cap ? nc : cap;
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nc)
        atomicAdd(&h[len_class(chunk_len(ends, k))], 1u);
    __syncthreads();
    if (threadIdx.x < kLenClasses && h[threadIdx.x])
        atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// hist[0..63] -> exclusive prefix in cursor[0..63] (one wave, serial in lane 0:
// 64 entries).
__global__ void k_chunk_class_scan(const uint32_t *__restrict__ hist,
                                   uint32_t *__restrict__ cursor)
{
    if (threadIdx.x != 0)
        return;
    uint32_t acc = 0;
    for (uint32_t c = 0; c < kLenClasses; c++) {
        cursor[c] = acc;
        acc += hist[c];
    }
}

// One chunk per lane: a slot in its class, reserved per workgroup.
__global__ __launch_bounds__(256) void k_chunk_scatter(const uint64_t *__restrict__ ends,
                                                       const uint64_t *__restrict__ n_chunks,
                                                       uint64_t cap, uint32_t *__restrict__ cursor,
                                                       uint32_t *__restrict__ order)
{
    __shared__ uint32_t cnt[kLenClasses], base[kLenClasses];
    if (threadIdx.x < kLenClasses)
        cnt[threadIdx.x] = 0;
    __syncthreads();
    uint64_t nc = *n_chunks;
    nc = nc < cap ? nc : cap;
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t cls = 0, local = 0;
    if (k < nc) {
        cls = len_class(chunk_len(ends, k));
        local = atomicAdd(&cnt[cls], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kLenClasses && cnt[threadIdx.x])
        base[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], cnt[threadIdx.x]);
    __syncthreads();
    if (k < nc)
        order[base[cls] + local] = (uint32_t)k;
}

// ------------------------------------------------------- one-launch finish
// For an input of up to kFinishTiles tiles, one workgroup does what follows
// the walk: verification, the serial repair, the scan of the tiles' counts,
// the packing of the ends and, when `order` is given, the length-class
// counting sort of the chunks.  A small chunking job then issues three
// launches (candidates, walk, finish) instead of eleven, each of which would
// cost a few microseconds of serial time.
constexpr uint32_t kFinishTiles = 1024;     // one thread per tile
constexpr uint64_t kFinishOrderCap = 65536; // chunks the workgroup orders

__global__ __launch_bounds__(1024) void k_sel_finish(SelArgs a, uint64_t *__restrict__ n_chunks,
                                                     uint64_t *__restrict__ ends, uint64_t cap,
                                                     uint32_t *__restrict__ order, uint64_t ocap)
{
    __shared__ uint32_t s_bad;
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t cls_n[kLenClasses];
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t == 0)
        s_bad = 0;
    if (t < kLenClasses)
        cls_n[t] = 0;
    __syncthreads();
    if (t >= 1 && t < a.n_tiles && a.exit_[t - 1] != a.first[t])
        atomicAdd(&s_bad, 1u);
    __syncthreads();
    if (s_bad) {
        if (t == 0) {
            for (uint32_t u = 1; u < a.n_tiles; u++) {
                const uint64_t entry = a.exit_[u - 1];
                if (entry != a.first[u])
                    walk_tile(a, u, entry);
            }
        }
        __syncthreads();
    }
    // exclusive scan of the tiles' start counts (the input is below 2^31
    // bytes, so the total fits 32 bits)
    const uint32_t c = t < a.n_tiles ? a.tcnt[t] : 0;
    const uint32_t x = wave_scan_incl(c, lane);
    if (lane == 63)
        wsum[wv] = x;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (uint32_t k = 0; k < 16; k++) {
        before += k < wv ? wsum[k] : 0;
        total += wsum[k];
    }
    // start number j >= 1 is end j-1; the last end is n
    emit_tile(a, t, c, before + x - c, ends, cap);
    const uint64_t m = total;
    if (t == 0) {
        if (m >= 1 && m - 1 < cap)
            ends[m - 1] = a.n;
        *n_chunks = m;
    }
    if (order == nullptr)
        return;
    __syncthreads(); // the ends above are visible to the whole workgroup
    const uint64_t nc = m < ocap ? m : ocap;
    for (uint64_t k = t; k < nc; k += 1024)
        atomicAdd(&cls_n[len_class(chunk_len(ends, k))], 1u);
    __syncthreads();
    if (wv == 0) {
        const uint32_t v = cls_n[lane];
        const uint32_t y = wave_scan_incl(v, lane);
        cls_n[lane] = y - v; // first slot of the class
    }
    __syncthreads();
    for (uint64_t k = t; k < nc; k += 1024)
        order[atomicAdd(&cls_n[len_class(chunk_len(ends, k))], 1u)] = (uint32_t)k;
}

static inline uint32_t nblk(uint64_t n, uint32_t b) { return (uint32_t)((n + b - 1) / b); }

hipError_t launch_cdc_candidates(const uint8_t *in, const CdcGeom &g, const CdcParams &p,
                                 uint8_t *ws, hipStream_t s)
{
    if (g.n == 0)
        return hipSuccess;
    uint64_t *l1 = reinterpret_cast<uint64_t *>(ws + g.off_l1);
    uint64_t *l2 = reinterpret_cast<uint64_t *>(ws + g.off_l2);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(ws + g.off_cnt);
    const uint32_t lgk = roll_lanes_log2(g.n_ranges);
    const dim3 grid(nblk(g.n_ranges << lgk, 256)), block(256);
    if (p.mask_bits <= 15) {
        const uint32_t b16 = (uint32_t)(p.base & 0xffffu);
        const uint32_t nb48 = (uint32_t)((0ull - p.b48) & 0xffffu);
        const uint32_t m = (uint32_t)(p.mask & 0xffffu);
        hipLaunchKernelGGL(k_cdc_roll_x2, grid, block, 0, s, in, g.n, b16, nb48,
                           m | (m << 16), l1, l2, cnt, lgk);
    } else if (p.mask_bits <= 32)
        hipLaunchKernelGGL((k_cdc_roll<uint32_t, 0>), grid, block, 0, s, in, g.n, p.base,
                           p.b48, p.mask, l1, l2, cnt, (uint64_t *)nullptr, lgk);
    else
        hipLaunchKernelGGL((k_cdc_roll<uint64_t, 0>), grid, block, 0, s, in, g.n, p.base,
                           p.b48, p.mask, l1, l2, cnt, (uint64_t *)nullptr, lgk);
    return hipGetLastError();
}

hipError_t launch_cdc_compact(const CdcGeom &g, uint8_t *ws, uint64_t *d_count,
                              uint64_t *d_cand, uint64_t cap, hipStream_t s)
{
    if (g.n == 0) {
        hipLaunchKernelGGL(k_store_zero_u64, dim3(1), dim3(64), 0, s, d_count);
        return hipGetLastError();
    }
    uint64_t *l1 = reinterpret_cast<uint64_t *>(ws + g.off_l1);
    uint64_t *l2 = reinterpret_cast<uint64_t *>(ws + g.off_l2);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(ws + g.off_cnt);
    uint64_t *rscan = reinterpret_cast<uint64_t *>(ws + g.off_rscan);
    hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, s, cnt, g.n_ranges, rscan, d_count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || d_cand == nullptr)
        return e;
    hipLaunchKernelGGL(k_cdc_compact, dim3(nblk(g.n_ranges, 256)), dim3(256), 0, s, l1, l2,
                       rscan, g.n_ranges, d_cand, cap);
    return hipGetLastError();
}

hipError_t launch_cdc_select(const CdcGeom &g, const CdcParams &p, uint8_t *ws,
                             uint64_t *d_n_chunks, uint64_t *d_ends, uint64_t cap,
                             hipStream_t s, const uint32_t **order)
{
    if (order)
        *order = nullptr;
    if (g.n == 0) {
        hipLaunchKernelGGL(k_store_zero_u64, dim3(1), dim3(64), 0, s, d_n_chunks);
        return hipGetLastError();
    }
    SelArgs a;
    a.l1 = reinterpret_cast<const uint64_t *>(ws + g.off_l1);
    a.l2 = reinterpret_cast<const uint64_t *>(ws + g.off_l2);
    a.n = g.n;
    a.min_len = p.min_len;
    a.max_len = p.max_len;
    a.tile_bytes = g.tile_bytes;
    a.warm_bytes = g.warm_bytes;
    a.n_tiles = g.n_tiles;
    a.tile_cap = g.tile_cap;
    a.exit_ = reinterpret_cast<uint64_t *>(ws + g.off_exit);
    a.first = reinterpret_cast<uint64_t *>(ws + g.off_first);
    a.tcnt = reinterpret_cast<uint32_t *>(ws + g.off_tcnt);
    a.starts = reinterpret_cast<uint64_t *>(ws + g.off_starts);
    a.flags = reinterpret_cast<uint32_t *>(ws + g.off_flags);
    a.bad = reinterpret_cast<uint32_t *>(ws + g.off_bad);
    uint64_t *toff = reinterpret_cast<uint64_t *>(ws + g.off_toff);
    uint64_t *total = reinterpret_cast<uint64_t *>(ws + g.off_misc);
    hipError_t e;
    if (g.n_tiles <= kFinishTiles && g.n < (1ull << 31)) {
        // the finisher orders the chunks too when they are few enough
        const uint64_t ocap = cap < g.ord_cap ? cap : g.ord_cap;
        uint32_t *ord = nullptr;
        if (order && ocap > 0 && ocap <= kFinishOrderCap)
            ord = reinterpret_cast<uint32_t *>(ws + g.off_ord);
        hipLaunchKernelGGL(k_sel_walk, dim3(g.n_tiles), dim3(64), 0, s, a);
        hipLaunchKernelGGL(k_sel_finish, dim3(1), dim3(1024), 0, s, a, d_n_chunks, d_ends, cap,
                           ord, ocap);
        e = hipGetLastError();
        if (e != hipSuccess || !order)
            return e;
        if (ord) {
            *order = ord;
            return hipSuccess;
        }
        return launch_chunk_order(g, ws, d_n_chunks, d_ends, cap, order, s);
    }
    // the packing kernel also counts the chunks per length class when the
    // order is wanted
    const uint64_t ocap = cap < g.ord_cap ? cap : g.ord_cap;
    uint32_t *hist = order && ocap > 0 ? reinterpret_cast<uint32_t *>(ws + g.off_hist) : nullptr;
    hipLaunchKernelGGL(k_sel_walk, dim3(g.n_tiles), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_sel_verify_scan, dim3(1), dim3(1024), 0, s, a, toff, total, hist);
    hipLaunchKernelGGL(k_sel_emit, dim3(nblk(g.n_tiles, 64)), dim3(64), 0, s, a, toff, total,
                       d_n_chunks, d_ends, cap, hist, ocap);
    e = hipGetLastError();
    if (e != hipSuccess || !hist)
        return e;
    uint32_t *cursor = hist + kLenClasses;
    uint32_t *ord = reinterpret_cast<uint32_t *>(ws + g.off_ord);
    hipLaunchKernelGGL(k_chunk_class_scan, dim3(1), dim3(64), 0, s, hist, cursor);
    hipLaunchKernelGGL(k_chunk_scatter, dim3(nblk(ocap, 256)), dim3(256), 0, s, d_ends,
                       d_n_chunks, ocap, cursor, ord);
    e = hipGetLastError();
    if (e == hipSuccess)
        *order = ord;
    return e;
}

hipError_t launch_chunk_order(const CdcGeom &g, uint8_t *ws, const uint64_t *d_n_chunks,
                              const uint64_t *d_ends, uint64_t cap, const uint32_t **order,
                              hipStream_t s)
{
    *order = nullptr;
    const uint64_t m = cap < g.ord_cap ? cap : g.ord_cap;
    if (g.n == 0 || m == 0)
        return hipSuccess;
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws + g.off_hist);
    uint32_t *cursor = hist + kLenClasses;
    uint32_t *ord = reinterpret_cast<uint32_t *>(ws + g.off_ord);
    hipError_t e = launch_zero_u32(hist, kLenClasses, s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_chunk_hist, dim3(nblk(m, 256)), dim3(256), 0, s, d_ends, d_n_chunks,
                       m, hist);
    hipLaunchKernelGGL(k_chunk_class_scan, dim3(1), dim3(64), 0, s, hist, cursor);
    hipLaunchKernelGGL(k_chunk_scatter, dim3(nblk(m, 256)), dim3(256), 0, s, d_ends,
                       d_n_chunks, m, cursor, ord);
    e = hipGetLastError();
    if (e == hipSuccess)
        *order = ord;
    return e;
}

hipError_t launch_window_hash(const uint8_t *in, uint64_t n, uint64_t base, uint64_t *w,
                              hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    uint64_t b48 = 1;
    for (int i = 0; i < 48; i++)
        b48 *= base;
    const uint64_t nr = (n + kRangeBytes - 1) / kRangeBytes;
    // the same split of ranges into parts as the candidate launch, so the
    // full-hash dump checks every part's warm-up
    const uint32_t lgk = roll_lanes_log2(nr);
    hipLaunchKernelGGL((k_cdc_roll<uint64_t, 1>), dim3(nblk(nr << lgk, 256)), dim3(256), 0, s,
                       in, n, base, b48, ~0ull, (uint64_t *)nullptr, (uint64_t *)nullptr,
                       (uint32_t *)nullptr, w, lgk);
    return hipGetLastError();
}

} // namespace crystal
