/*
 * tinymt_device.h -- device-side TinyMT32 streams for user kernels.
 *
 * The paper's hybrid for TinyMT (sec. 4.2): the threads of a group share one
 * parameter set and each thread draws from its own sub-stream of that
 * generator, the sequence being cut into chunks of 2^64 outputs (sequence
 * splitting, sec. 2.3).  A TinyMT stream set (mrg_streamset_create_tinymt)
 * holds, per stream, six state words (s0, s1, s2, s3, q, 0) -- q the global
 * index of its parameter set -- and, per parameter set, a record of
 * tmt::kRecordWords words (parameters, characteristic polynomial, jump
 * table; layout in tinymt_arith.hpp).  Records are stored for sets
 * q0, q0 + 1, ... (mrg_streamset_tinymt_info gives q0 and their address).
 *
 * Usage (one stream per thread):
 *
 *   mrg::TinyMTStream s;
 *   s.load(planes, n_streams, i, records, q0);
 *   float u = s.next_f32();
 *   s.jump(1000);                     // optional: 1000 outputs ahead
 *   s.store(planes, n_streams, i);
 *
 * Draws equal mrg_fill's: value k here is value k of row i of a
 * stream-major fill from the same state.  uint32 outputs are the tempered
 * words; FP32 (2 * (w >> 9) + 1) * 2^-24 and FP64 (2w + 1) * 2^-33, exact
 * and in (0, 1).  Header-only; include from HIP device code.
 *
 * Parity unpinned: no known-answer output of TinyMT32 was available, so the
 * transition, tempering and seeding rest on their written definition; the
 * library's outputs equal the oracle's bit for bit.
 */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tinymt_arith.hpp"

namespace mrg {

struct TinyMTStream {
    uint32_t s0, s1, s2, s3;   // the state (bit 31 of s0 outside it)
    uint32_t q;                // global index of the parameter set
    uint32_t mat1, mat2, tmat; // the set's parameters
    const uint32_t *rec;       // the set's record
    // draws are exact as they come (no cheaper checked form)
    static constexpr bool kCheckedDraws = false;

    // Stream i of a set whose six state planes of n_streams words start at
    // planes; records of the sets q0, q0 + 1, ...
    __device__ __forceinline__ void load(const uint32_t *planes, uint64_t n_streams, uint64_t i,
                                         const uint32_t *records, uint64_t q0)
    {
        s0 = planes[i];
        s1 = planes[n_streams + i];
        s2 = planes[2 * n_streams + i];
        s3 = planes[3 * n_streams + i];
        q = planes[4 * n_streams + i];
        rec = records + (uint64_t)(q - q0) * tmt::kRecordWords;
        mat1 = rec[0];
        mat2 = rec[1];
        tmat = rec[2];
    }
    // Write the state words back (the parameter set does not change).
    __device__ __forceinline__ void store(uint32_t *planes, uint64_t n_streams, uint64_t i) const
    {
        planes[i] = s0;
        planes[n_streams + i] = s1;
        planes[2 * n_streams + i] = s2;
        planes[3 * n_streams + i] = s3;
    }
    __device__ __forceinline__ uint32_t next_u32()
    {
        tmt::step(s0, s1, s2, s3, mat1, mat2);
        return tmt::temper(s0, s2, s3, tmat);
    }
    __device__ __forceinline__ float next_f32()
    {
        // 1 + k * 2^-23 minus 1 - 2^-24 is (2k + 1) * 2^-24, exactly
        return __uint_as_float(0x3F800000u | (next_u32() >> 9)) - 0x1.fffffep-1f;
    }
    __device__ __forceinline__ double next_f64()
    {
        return __fma_rn((double)next_u32(), 0x1p-32, 0x1p-33);  // (2w + 1) * 2^-33, exact
    }
    // Move e = e0 + e1 * 2^64 + e2 * 2^128 outputs ahead (polynomial jump
    // with the set's table).
    __device__ __forceinline__ void jump(uint64_t e0, uint64_t e1 = 0, uint64_t e2 = 0)
    {
        uint32_t s[4] = {s0, s1, s2, s3};
        tmt::jump(s, mat1, mat2, rec + tmt::kRecPhi, rec + tmt::kRecPow, e0, e1, e2);
        s0 = s[0];
        s1 = s[1];
        s2 = s[2];
        s3 = s[3];
    }
};

}  // namespace mrg
