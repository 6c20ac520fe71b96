// Minimal matrix generator (sigma-basis, Section 2.4) and rank read-out
// (Section 2.5, steps 3-4) on the host.  Internal C++.
#pragma once
#include <stdint.h>

#include <vector>

#include "engine.h"

namespace bwr {

// s x s polynomial matrix, entry (r, c) stored contiguously: a[(r * cols + c) * len + k]
struct PolyMat {
    int rows = 0, cols = 0;
    int64_t len = 0;  // number of coefficients per entry
    std::vector<uint32_t> a;
    void resize(int r, int c, int64_t l) {
        rows = r;
        cols = c;
        len = l;
        a.assign((size_t)r * c * (size_t)l, 0u);
    }
    uint32_t* at(int r, int c) { return a.data() + ((size_t)r * cols + c) * (size_t)len; }
    const uint32_t* at(int r, int c) const { return a.data() + ((size_t)r * cols + c) * (size_t)len; }
};

struct Generator {
    int s = 0;
    std::vector<int64_t> delta;  // shifted degrees of the chosen rows
    PolyMat P;                   // their p-parts (s x s); F_i(x) = x^delta_i P_i(1/x)
};

struct SigmaStats {
    double seconds = 0;
    int threads = 1;
};

// Sigma-basis of [S(x); -I_s] of order L (PM-Basis with M-Basis leaves) and
// the generator rows.  S: host array L x s x s (row-major per term), residues < p.
Error min_generator(const uint32_t* S, int64_t L, int32_t s, uint32_t p, Generator* out, SigmaStats* st = nullptr);

// Checks sum_j F_{i,j} S_{l+j} = 0 on the terms L .. L_total - 1 (beyond those
// the basis was built from).
Error check_generator(const Generator& g, const uint32_t* S, int64_t L, int64_t L_total, uint32_t p);

// rank = deg det F - codeg det F = deg det P - val_x det P.
Error rank_from_generator(const Generator& g, uint32_t p, int64_t* rank);

// Plain M-Basis only (for tests of the divide and conquer against the leaf).
Error min_generator_mbasis(const uint32_t* S, int64_t L, int32_t s, uint32_t p, Generator* out);

// Polynomial matrix product window [lo, hi) of A * B mod p via NTT + CRT (exposed for tests).
void polymat_mul(const PolyMat& A, const PolyMat& B, int64_t lo, int64_t hi, uint32_t p, PolyMat* C);

// Twiddle tables of FFT prime t (0: 2013265921, 1: 1811939329, 2: 2113929217)
// for transforms up to 2^lg points, copied into the caller's arrays of 2^lg
// entries each: tw[half + j] = w_{2 half}^j, with Shoup constants, and the
// same for the inverse roots.  Safe beside concurrent products.
void ntt_tables(int t, int lg, uint32_t* q, uint32_t* tw, uint32_t* tws, uint32_t* itw, uint32_t* itws);

void set_sigma_threads(int n);
int sigma_threads();

}  // namespace bwr
