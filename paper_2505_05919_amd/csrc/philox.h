// Philox4x32-10 for the device (included inside the kernels' namespace).
#pragma once

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The key words are
// wave-uniform (the chain's seed), so the key schedule lives in SGPRs.  From
// the third round on every counter word is per-lane and each round is two
// v_mad_u64_u32 and two v_bitop3_b32 (truth table 0x96 = a ^ b ^ c).
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
        uint32_t n0, n2;
        if (r < 2) {                                    // c1 (and c2, c3) may still be uniform
            n0 = hi1 ^ (c1 ^ k0);
            n2 = hi0 ^ (c3 ^ k1);
        } else {                                        // 3-input XOR in one v_bitop3_b32
            n0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
            n2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
        }
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return make_uint4(c0, c1, c2, c3);
}

