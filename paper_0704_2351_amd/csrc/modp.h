// Arithmetic in GF(p) for primes 3 <= p < 2^31, shared by host and device code.
//
// Residues are uint32 in [0, p).  Reductions use Barrett's method with a
// precomputed reciprocal: for x < 2^64 and mu64 = floor(2^64 / p),
// q = floor(x * mu64 / 2^64) is floor(x / p) or one less, so x - q p lies in
// [0, 2p) and one conditional subtraction finishes (likewise for 32-bit x with
// mu32 = floor(2^32 / p)).  The sequence of Section 2.2 is exact arithmetic
// modulo p; these helpers are the only place a reduction happens.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__) || defined(__HIP__)
#define BWR_HD __host__ __device__ __forceinline__
#else
#define BWR_HD inline
#endif

namespace bwr {

struct ModP {
    uint32_t p;
    uint32_t mu32;  // floor(2^32 / p)
    uint64_t mu64;  // floor(2^64 / p)

    static ModP make(uint32_t prime) {
        ModP m;
        m.p = prime;
        m.mu32 = (uint32_t)((((uint64_t)1) << 32) / prime);
        // floor(2^64 / p) computed without 128-bit types: 2^64 = (2^64 - 1) + 1
        uint64_t q = UINT64_MAX / prime;
        uint64_t r = UINT64_MAX - q * prime;  // (2^64 - 1) mod p
        if (r + 1 == prime) q += 1;
        m.mu64 = q;
        return m;
    }
};

BWR_HD uint64_t umulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

// x mod p for any 64-bit x
BWR_HD uint32_t red64(const ModP& m, uint64_t x) {
    uint64_t q = umulhi64(x, m.mu64);
    uint64_t r = x - q * (uint64_t)m.p;
    return (uint32_t)(r >= m.p ? r - m.p : r);
}

// x mod p for any 32-bit x
BWR_HD uint32_t red32(const ModP& m, uint32_t x) {
    uint32_t q = (uint32_t)(((uint64_t)x * m.mu32) >> 32);
    uint32_t r = x - q * m.p;
    return r >= m.p ? r - m.p : r;
}

// signed 32-bit value mod p, result in [0, p)
BWR_HD uint32_t reds32(const ModP& m, int32_t x) {
    uint32_t a = x < 0 ? (uint32_t)(-(int64_t)x) : (uint32_t)x;
    uint32_t r = red32(m, a);
    return (x < 0 && r) ? m.p - r : r;
}

// signed 64-bit value mod p, result in [0, p)
BWR_HD uint32_t reds64(const ModP& m, int64_t x) {
    uint64_t a = x < 0 ? (uint64_t)0 - (uint64_t)x : (uint64_t)x;
    uint32_t r = red64(m, a);
    return (x < 0 && r) ? m.p - r : r;
}

// a * b mod p for residues a, b
BWR_HD uint32_t mulmod(const ModP& m, uint32_t a, uint32_t b) {
    return red64(m, (uint64_t)a * b);
}

// a * b mod p when p <= 2^16 (the product fits 32 bits)
BWR_HD uint32_t mulmod16(const ModP& m, uint32_t a, uint32_t b) {
    return red32(m, a * b);
}

BWR_HD uint32_t addmod(const ModP& m, uint32_t a, uint32_t b) {
    uint32_t s = a + b;
    return s >= m.p ? s - m.p : s;
}

BWR_HD uint32_t powmod(const ModP& m, uint32_t a, uint64_t e) {
    uint32_t r = 1 % m.p;
    while (e) {
        if (e & 1) r = mulmod(m, r, a);
        a = mulmod(m, a, a);
        e >>= 1;
    }
    return r;
}

BWR_HD uint32_t invmod(const ModP& m, uint32_t a) { return powmod(m, a, m.p - 2); }

}  // namespace bwr
