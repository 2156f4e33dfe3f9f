/*
 * Seeded synthetic-input generators.
 *
 * This file holds NO hashing arithmetic: it only produces input bytes and
 * random draws, which both the CPU oracle and the GPU path consume.  The
 * random source is SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), a counter-based generator:
 * output k of a generator seeded with s is mix(s + (k+1)*GOLDEN), where mix is
 * the variant-13 64-bit finaliser from that paper.
 *
 * Byte streams are the generator's 64-bit outputs written little-endian, the
 * last word truncated at the end of the buffer.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>

#define GEN_GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t gen_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Output k (0-based) of the generator seeded with `seed`. */
uint64_t gen_splitmix64_at(uint64_t seed, uint64_t k)
{
    return gen_mix(seed + (k + 1) * GEN_GOLDEN);
}

/* n consecutive outputs, starting at output `first`. */
void gen_u64(uint64_t seed, uint64_t first, uint64_t *out, size_t n)
{
    for (size_t i = 0; i < n; i++)
        out[i] = gen_mix(seed + (first + i + 1) * GEN_GOLDEN);
}

/* Fill n bytes: output k supplies bytes [8k, 8k+8), little-endian. */
void gen_bytes(uint64_t seed, uint8_t *out, size_t n)
{
    size_t words = n / 8, i;
    for (i = 0; i < words; i++) {
        uint64_t w = gen_mix(seed + (i + 1) * GEN_GOLDEN);
        memcpy(out + 8 * i, &w, 8); /* host is little-endian (x86-64) */
    }
    size_t rem = n - 8 * words;
    if (rem) {
        uint64_t w = gen_mix(seed + (words + 1) * GEN_GOLDEN);
        for (size_t b = 0; b < rem; b++)
            out[8 * words + b] = (uint8_t)(w >> (8 * b));
    }
}

/*
 * Many independent byte streams into one arena: stream j fills
 * out[off[j], off[j]+len[j]) from seed seeds[j].  Used for job sets and for the
 * batched-buffer arena.
 */
void gen_bytes_multi(const uint64_t *seeds, const uint64_t *off,
                     const uint64_t *len, size_t n_streams, uint8_t *out)
{
    for (size_t j = 0; j < n_streams; j++)
        gen_bytes(seeds[j], out + off[j], (size_t)len[j]);
}
