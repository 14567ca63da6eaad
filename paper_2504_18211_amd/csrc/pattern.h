/*
 * pattern.h -- the seeded payload words written into blocks and checked on
 * read-back (the paper's driver writes data into every block it allocates
 * and checks it, Methods).  Word j of request i under seed s is
 *     fmix32(s ^ fmix32(i) ^ j * 0x9E3779B9),
 * fmix32 being the 32-bit finaliser of MurmurHash3 (public domain); a block
 * of n bytes holds the first n bytes of that little-endian word sequence.
 * Internal to the HIP library (kernels of hbheap.hip, growth.hip, serve.hip).
 */
#ifndef HBHEAP_PATTERN_H
#define HBHEAP_PATTERN_H

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint32_t fmix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}
__device__ __forceinline__ uint32_t pat_word(uint32_t sr, uint32_t j) { return fmix32(sr ^ (j * 0x9E3779B9u)); }

/* Bytes [b0, b1) of the block, b0 a multiple of 16; `step` 16-byte units
 * apart per iteration starting at unit `first`. */
__device__ __forceinline__ void pat_write_range(uint8_t* p, uint64_t size, uint32_t sr, uint64_t first, uint64_t step)
{
    const uint64_t nq = size >> 4;
    uint4* q = (uint4*)p;
    for (uint64_t u = first; u < nq; u += step) {
        const uint32_t j = (uint32_t)(u * 4);
        q[u] = make_uint4(pat_word(sr, j), pat_word(sr, j + 1), pat_word(sr, j + 2), pat_word(sr, j + 3));
    }
    if (first == 0) {
        for (uint64_t b = nq << 4; b < size; ++b) {
            const uint32_t w = pat_word(sr, (uint32_t)(b >> 2));
            p[b] = (uint8_t)(w >> (8 * (b & 3)));
        }
    }
}

__device__ __forceinline__ uint32_t pat_check_range(const uint8_t* p, uint64_t size, uint32_t sr, uint64_t first, uint64_t step)
{
    const uint64_t nq = size >> 4;
    const uint4* q = (const uint4*)p;
    uint32_t bad = 0;
    for (uint64_t u = first; u < nq; u += step) {
        const uint32_t j = (uint32_t)(u * 4);
        const uint4 v = q[u];
        bad += (v.x != pat_word(sr, j)) + (v.y != pat_word(sr, j + 1)) + (v.z != pat_word(sr, j + 2)) +
               (v.w != pat_word(sr, j + 3));
    }
    if (first == 0) {
        /* tail bytes, counted per (partial) word */
        for (uint64_t b = nq << 4; b < size; b += 4) {
            const uint32_t w = pat_word(sr, (uint32_t)(b >> 2));
            bool ok = true;
            for (uint64_t e = b; e < size && e < b + 4; ++e) ok &= p[e] == (uint8_t)(w >> (8 * (e & 3)));
            bad += ok ? 0u : 1u;
        }
    }
    return bad;
}

}  // namespace

#endif
