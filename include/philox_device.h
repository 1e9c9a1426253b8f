/*
 * philox_device.h -- device-side Philox4x32-10 streams for user kernels.
 *
 * The counter-based generator of Salmon, Moraes, Dror & Shaw (SC 2011), the
 * second family the library provides (mrg_streamset_create_philox).  A
 * stream's six state words are (position lo, hi, stream id lo, hi, key lo,
 * hi); its output number p is word p % 4 of the ten-round block whose counter
 * is (p / 4 as two words, stream id as two words), under the key.  Positions
 * wrap at 2^64, so block numbers wrap at 2^62.
 *
 * Usage (one stream per thread, the planes of a Philox stream set from
 * mrg_streamset_states_ptr):
 *
 *   mrg::PhiloxStream s;
 *   s.load(planes, n_streams, i);
 *   float u = s.next_f32();
 *   s.store(planes, n_streams, i);   // only the position changes
 *
 * Conversions match the library's fills: uint32 words as they are; FP32
 * (2*(w >> 9) + 1) * 2^-24 and FP64 (2*w + 1) * 2^-33, exact and in (0, 1).
 * Header-only; include from HIP device code.
 *
 * Parity unpinned: the round multipliers below are typed from the published
 * definition and no known-answer vector was available to check them; the
 * Weyl increments, the round wiring, the key schedule and the round count
 * are pinned, and the library's outputs equal the oracle's bit for bit.
 */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrg {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;  // round multipliers
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;  // Weyl key increments: 2^32 (sqrt 5 - 1) / 2,
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;  //                       2^32 (sqrt 3 - 1)

// Ten rounds on the counter c under the key (k0, k1): each round multiplies
// words 0 and 2 by the multipliers, keeps the low halves as the new words 3
// and 1 and xors the high halves with words 1 and 3 and the round key into
// the new words 0 and 2; the round key moves by the Weyl increments.
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c[0];
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
}

// The 4 words of block b of the stream with state words w (id w[2..3], key
// w[4..5]).
__device__ __forceinline__ void philox_block(const uint32_t *w, uint64_t b, uint32_t out[4])
{
    b &= ((uint64_t)1 << 62) - 1;
    out[0] = (uint32_t)b;
    out[1] = (uint32_t)(b >> 32);
    out[2] = w[2];
    out[3] = w[3];
    philox10(out, w[4], w[5]);
}

__device__ __forceinline__ float philox_to_f32(uint32_t w)
{
    return __uint_as_float(0x3F800000u | (w >> 9)) - 0x1.fffffep-1f;  // exact
}

__device__ __forceinline__ double philox_to_f64(uint32_t w)
{
    return __fma_rn((double)w, 0x1p-32, 0x1p-33);  // exact
}

// One Philox stream drawn by one thread.  The block of the current position
// is kept, so four consecutive draws cost one ten-round block.
struct PhiloxStream {
    uint32_t w[6];
    uint32_t blk[4];
    uint64_t cached = ~(uint64_t)0;  // block number held in blk

    // Stream i of a set whose six state planes of n_streams words start at planes.
    __device__ __forceinline__ void load(const uint32_t *planes, uint64_t n_streams, uint64_t i)
    {
#pragma unroll
        for (int c = 0; c < 6; ++c) w[c] = planes[c * n_streams + i];
        cached = ~(uint64_t)0;
    }
    // Write the position back (the id and key do not change).
    __device__ __forceinline__ void store(uint32_t *planes, uint64_t n_streams, uint64_t i) const
    {
        planes[i] = w[0];
        planes[n_streams + i] = w[1];
    }
    __device__ __forceinline__ uint64_t position() const
    {
        return (uint64_t)w[0] | (uint64_t)w[1] << 32;
    }
    // Move e outputs ahead (e mod 2^64).
    __device__ __forceinline__ void jump(uint64_t e)
    {
        const uint64_t p = position() + e;
        w[0] = (uint32_t)p;
        w[1] = (uint32_t)(p >> 32);
    }
    __device__ __forceinline__ uint32_t next_u32()
    {
        const uint64_t p = position();
        const uint64_t b = (p >> 2) & (((uint64_t)1 << 62) - 1);
        if (b != cached) {
            philox_block(w, b, blk);
            cached = b;
        }
        jump(1);
        const uint32_t j = (uint32_t)p & 3u;  // select, not index (keeps blk in registers)
        const uint32_t lo = j & 1u ? blk[1] : blk[0];
        const uint32_t hi = j & 1u ? blk[3] : blk[2];
        return j & 2u ? hi : lo;
    }
    __device__ __forceinline__ float next_f32() { return philox_to_f32(next_u32()); }
    __device__ __forceinline__ double next_f64() { return philox_to_f64(next_u32()); }
};

}  // namespace mrg
