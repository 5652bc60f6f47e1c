// Philox4x32-10 for the device (included inside the kernels' namespace).
#pragma once

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The key words are
// wave-uniform (the chain's seed), so the key schedule lives in SGPRs.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mulhilo(uint32_t m, uint32_t x, uint32_t& hi, uint32_t& lo)
{
    const uint64_t p = (uint64_t)m * (uint64_t)x;     // one v_mad_u64_u32
    hi = (uint32_t)(p >> 32);
    lo = (uint32_t)p;
}

__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo(0xD2511F53u, c0, hi0, lo0);
        mulhilo(0xCD9E8D57u, c2, hi1, lo1);
        const uint32_t n0 = hi1 ^ (c1 ^ k0);
        const uint32_t n2 = hi0 ^ (c3 ^ k1);
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return make_uint4(c0, c1, c2, c3);
}

