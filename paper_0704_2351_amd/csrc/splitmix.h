// Counter-based SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), host and device.
//
// The random blocks of step 2 of the rank algorithm (Section 2.5) and the
// diagonal preconditioners are drawn from it:
//   output(state, i)   = mix(state + (i + 1) * gamma)
//   element(seed,t,i)  = output(output(seed, t), i)
// with stream t = 0 for V, 1 for U, 2 for the row diagonal, 3 for the column
// diagonal.  Block entries take h mod p; diagonal entries take 1 + h mod (p-1).
// Counter-based, so any element can be regenerated anywhere from (seed, t, i).
#pragma once
#include <stdint.h>

#include "modp.h"

namespace bwr {

enum : int { STREAM_V = 0, STREAM_U = 1, STREAM_DROW = 2, STREAM_DCOL = 3 };

constexpr uint64_t SM_GAMMA = 0x9E3779B97F4A7C15ull;

BWR_HD uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

BWR_HD uint64_t sm_output(uint64_t state, uint64_t i) { return sm_mix(state + (i + 1) * SM_GAMMA); }

BWR_HD uint64_t sm_key(uint64_t seed, int stream) { return sm_output(seed, (uint64_t)stream); }

// residue in [0, p) (diag = 0) or in [1, p - 1] (diag = 1)
BWR_HD uint32_t sm_residue(const ModP& m, uint64_t key, uint64_t i, int diag) {
    uint64_t h = sm_output(key, i);
    if (diag) return 1u + (uint32_t)(h % (uint64_t)(m.p - 1));
    return (uint32_t)(h % (uint64_t)m.p);
}

}  // namespace bwr
