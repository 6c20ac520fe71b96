// Sigma-basis (PM-Basis of Giorgi, Jeannerod and Villard, the algorithm named
// in Section 2.4) and the rank read-out of Section 2.5, on the host.
//
// Approximation problem: G(x) = [S(x); -I_s] (2s x s), S(x) = sum_{k<L} S_k x^k.
// An order-L sigma-basis P (2s x 2s) has P G = 0 mod x^L and is minimal for the
// shift (0^s, 1^s): a row [p, r] has shifted degree max(deg p, deg r + 1).
// PM-Basis halves the order: P1 = basis of order L/2, G2 = (P1 G) x^{-L/2},
// P2 = basis of G2 of order L - L/2, P = P2 P1.  Products of polynomial
// matrices go through number-theoretic transforms modulo three 31-bit FFT
// primes c 2^k + 1 and the Chinese remainder theorem, with prod q_i larger than
// (inner dimension) x (length) x p^2 (Section 2.4 on FFT primes and CRT).
// Leaves (small order) use the iterative M-Basis.
//
// Generator: the s basis rows of smallest shifted degree (ties: row index);
// F_i(x) = x^delta_i p_i(1/x).  Read-out: with det F(x) = x^{sum delta} det P(1/x),
// deg det F - codeg det F = deg det P - val det P = sum delta - val det F - val det P;
// both valuations come from local Smith forms over GF(p)[[x]] truncated at x^K
// (the low coefficients only, as Section 2.5 suggests).
#include "sigma.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <shared_mutex>
#include <thread>

namespace bwr {

// ------------------------------------------------------------------ thread pool
namespace {

class Pool {
   public:
    explicit Pool(int n) { start(n); }
    ~Pool() { stop(); }
    int size() const { return (int)workers_.size() + 1; }
    void resize(int n) {
        stop();
        start(n);
    }
    // runs fn(i) for i in [0, n) on all threads; returns when done.  Calls from several host threads
    // take turns (one job at a time).
    void run(int64_t n, const std::function<void(int64_t)>& fn) {
        if (n <= 0) return;
        if (workers_.empty() || n == 1) {
            for (int64_t i = 0; i < n; ++i) fn(i);
            return;
        }
        std::lock_guard<std::mutex> turn(run_mu_);
        std::unique_lock<std::mutex> lk(mu_);
        job_ = &fn;
        total_ = n;
        next_.store(0);
        active_ = (int)workers_.size();
        ++gen_;
        cv_.notify_all();
        lk.unlock();
        work();
        lk.lock();
        done_cv_.wait(lk, [&] { return active_ == 0; });
        job_ = nullptr;
    }

   private:
    void work() {
        const std::function<void(int64_t)>* fn = job_;
        for (;;) {
            int64_t i = next_.fetch_add(1);
            if (i >= total_) break;
            (*fn)(i);
        }
    }
    void start(int n) {
        quit_ = false;
        for (int t = 1; t < n; ++t)
            workers_.emplace_back([this] {
                uint64_t seen = 0;
                for (;;) {
                    std::unique_lock<std::mutex> lk(mu_);
                    cv_.wait(lk, [&] { return quit_ || gen_ != seen; });
                    if (quit_) return;
                    seen = gen_;
                    lk.unlock();
                    work();
                    lk.lock();
                    if (--active_ == 0) done_cv_.notify_all();
                }
            });
    }
    void stop() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            quit_ = true;
        }
        cv_.notify_all();
        for (auto& w : workers_) w.join();
        workers_.clear();
    }
    std::vector<std::thread> workers_;
    std::mutex mu_, run_mu_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(int64_t)>* job_ = nullptr;
    int64_t total_ = 0;
    std::atomic<int64_t> next_{0};
    int active_ = 0;
    uint64_t gen_ = 0;
    bool quit_ = false;
};

int default_threads() {
    unsigned h = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(h, 16u));
}

std::mutex g_pool_mu;
Pool& pool() {
    static Pool p(default_threads());
    return p;
}

// ------------------------------------------------------------------ NTT primes
struct NttPrime {
    uint32_t q = 0, g = 0;
    ModP mp;
    int max_log = 0;
    // per-level twiddles: tw[half + j] = w_len^j (len = 2 half), with Shoup constants
    std::vector<uint32_t> tw, tws, itw, itws;
    int table_log = 0;
};

uint32_t shoup_pre(uint32_t w, uint32_t q) { return (uint32_t)(((uint64_t)w << 32) / q); }

inline uint32_t mul_shoup(uint32_t a, uint32_t w, uint32_t wp, uint32_t q) {
    uint32_t qt = (uint32_t)(((uint64_t)a * wp) >> 32);
    uint32_t r = a * w - qt * q;
    return r >= q ? r - q : r;
}

uint32_t find_generator(uint32_t q) {
    ModP mp = ModP::make(q);
    uint32_t f = q - 1;
    std::vector<uint32_t> fac;
    for (uint32_t d = 2; (uint64_t)d * d <= f; ++d)
        if (f % d == 0) {
            fac.push_back(d);
            while (f % d == 0) f /= d;
        }
    if (f > 1) fac.push_back(f);
    for (uint32_t g = 2;; ++g) {
        bool ok = true;
        for (uint32_t d : fac)
            if (powmod(mp, g, (q - 1) / d) == 1) {
                ok = false;
                break;
            }
        if (ok) return g;
    }
}

NttPrime make_prime(uint32_t q) {
    NttPrime P;
    P.q = q;
    P.mp = ModP::make(q);
    P.g = find_generator(q);
    uint32_t e = q - 1;
    while (!(e & 1)) {
        e >>= 1;
        ++P.max_log;
    }
    return P;
}

// 2013265921 = 15 * 2^27 + 1, 1811939329 = 27 * 2^26 + 1, 2113929217 = 63 * 2^25 + 1
NttPrime g_primes[3];
std::once_flag g_primes_once;
// Growing a table reallocates it: growth takes this lock exclusively, and every use of the tables (the
// transforms of a product, a copy) holds it shared, so that read-out threads running sigma-bases side by
// side never read a table that another thread is replacing.
std::shared_mutex g_tw_rw;

void init_primes() {
    std::call_once(g_primes_once, [] {
        g_primes[0] = make_prime(2013265921u);
        g_primes[1] = make_prime(1811939329u);
        g_primes[2] = make_prime(2113929217u);
    });
}

void ensure_tables(NttPrime& P, int lg) {
    std::unique_lock<std::shared_mutex> lk(g_tw_rw);
    if (P.table_log >= lg) return;
    const size_t N = (size_t)1 << lg;
    P.tw.assign(N, 0);
    P.tws.assign(N, 0);
    P.itw.assign(N, 0);
    P.itws.assign(N, 0);
    for (int l = 1; l <= lg; ++l) {
        size_t half = (size_t)1 << (l - 1);
        uint32_t w = powmod(P.mp, P.g, (uint64_t)(P.q - 1) >> l);
        uint32_t wi = invmod(P.mp, w);
        uint32_t x = 1, xi = 1;
        for (size_t j = 0; j < half; ++j) {
            P.tw[half + j] = x;
            P.tws[half + j] = shoup_pre(x, P.q);
            P.itw[half + j] = xi;
            P.itws[half + j] = shoup_pre(xi, P.q);
            x = mulmod(P.mp, x, w);
            xi = mulmod(P.mp, xi, wi);
        }
    }
    P.table_log = lg;
}

// forward: decimation in frequency, natural order in, bit-reversed out
void ntt_dif(uint32_t* a, int lg, const NttPrime& P) {
    const uint32_t q = P.q;
    for (int l = lg; l >= 1; --l) {
        const size_t len = (size_t)1 << l, half = len >> 1;
        const uint32_t* w = P.tw.data() + half;
        const uint32_t* wp = P.tws.data() + half;
        for (size_t i = 0; i < ((size_t)1 << lg); i += len) {
            uint32_t* x = a + i;
            uint32_t* y = a + i + half;
            for (size_t j = 0; j < half; ++j) {
                uint32_t u = x[j], v = y[j];
                uint32_t s = u + v;
                x[j] = s >= q ? s - q : s;
                uint32_t d = u >= v ? u - v : u + q - v;
                y[j] = mul_shoup(d, w[j], wp[j], q);
            }
        }
    }
}

// inverse: decimation in time, bit-reversed in, natural order out (unscaled)
void ntt_dit_inv(uint32_t* a, int lg, const NttPrime& P) {
    const uint32_t q = P.q;
    for (int l = 1; l <= lg; ++l) {
        const size_t len = (size_t)1 << l, half = len >> 1;
        const uint32_t* w = P.itw.data() + half;
        const uint32_t* wp = P.itws.data() + half;
        for (size_t i = 0; i < ((size_t)1 << lg); i += len) {
            uint32_t* x = a + i;
            uint32_t* y = a + i + half;
            for (size_t j = 0; j < half; ++j) {
                uint32_t u = x[j];
                uint32_t v = mul_shoup(y[j], w[j], wp[j], q);
                uint32_t s = u + v;
                x[j] = s >= q ? s - q : s;
                y[j] = u >= v ? u - v : u + q - v;
            }
        }
    }
}

int ceil_log2(int64_t x) {
    int l = 0;
    while (((int64_t)1 << l) < x) ++l;
    return l;
}

// schoolbook window product for short operands
void mul_naive(const PolyMat& A, const PolyMat& B, int64_t lo, int64_t hi, const ModP& mp, PolyMat* C) {
    const int r = A.rows, k = A.cols, c = B.cols;
    C->resize(r, c, hi - lo);
    pool().run((int64_t)r * c, [&](int64_t idx) {
        int i = (int)(idx / c), l = (int)(idx % c);
        uint32_t* out = C->at(i, l);
        std::vector<uint64_t> lo32(hi - lo, 0), hi32(hi - lo, 0);
        for (int j = 0; j < k; ++j) {
            const uint32_t* a = A.at(i, j);
            const uint32_t* b = B.at(j, l);
            for (int64_t x = 0; x < A.len; ++x) {
                if (!a[x]) continue;
                int64_t y0 = std::max<int64_t>(0, lo - x), y1 = std::min<int64_t>(B.len, hi - x);
                for (int64_t y = y0; y < y1; ++y) {
                    uint64_t pr = (uint64_t)a[x] * b[y];
                    lo32[x + y - lo] += pr & 0xffffffffu;
                    hi32[x + y - lo] += pr >> 32;
                }
            }
        }
        const uint32_t r32 = red64(mp, (uint64_t)1 << 32);
        for (int64_t t = 0; t < hi - lo; ++t)
            out[t] = addmod(mp, red64(mp, lo32[t]), mulmod(mp, red64(mp, hi32[t]), r32));
    });
}

}  // namespace

void ntt_tables(int t, int lg, uint32_t* q, uint32_t* tw, uint32_t* tws, uint32_t* itw, uint32_t* itws) {
    init_primes();
    NttPrime& P = g_primes[t];
    ensure_tables(P, lg);
    std::shared_lock<std::shared_mutex> lk(g_tw_rw);
    const size_t n = (size_t)1 << lg;
    *q = P.q;
    std::memcpy(tw, P.tw.data(), n * 4);
    std::memcpy(tws, P.tws.data(), n * 4);
    std::memcpy(itw, P.itw.data(), n * 4);
    std::memcpy(itws, P.itws.data(), n * 4);
}

void set_sigma_threads(int n) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    pool().resize(std::max(1, n));
}
int sigma_threads() { return pool().size(); }

// ------------------------------------------------------------------ polynomial matrix product
void polymat_mul(const PolyMat& A, const PolyMat& B, int64_t lo, int64_t hi, uint32_t p, PolyMat* C) {
    const ModP mp = ModP::make(p);
    const int r = A.rows, k = A.cols, c = B.cols;
    const int64_t minlen = std::min(A.len, B.len);
    if (minlen <= 48 || (double)A.len * (double)B.len < 4096.0) {
        mul_naive(A, B, lo, hi, mp, C);
        return;
    }
    init_primes();
    // bound on each exact coefficient of the window: k * minlen * (p - 1)^2
    const double bound = (double)k * (double)minlen * (double)(p - 1) * (double)(p - 1);
    int np = 1;
    double prod = 2013265921.0;
    while (prod <= bound * 1.0001) {
        prod *= (double)g_primes[np].q;
        ++np;
        if (np == 3) break;
    }
    const int64_t need = std::max<int64_t>(hi, A.len + B.len - 1 - lo);
    const int lg = ceil_log2(need);
    const size_t N = (size_t)1 << lg;
    for (int t = 0; t < np; ++t) ensure_tables(g_primes[t], lg);
    // tables only grow, so they still cover 2^lg points; no table is replaced while this is held
    std::shared_lock<std::shared_mutex> tables(g_tw_rw);
    const int64_t W = hi - lo;
    // residues of the window for each prime: res[t][(i*c+l)*W + x]
    std::vector<std::vector<uint32_t>> res(np, std::vector<uint32_t>((size_t)r * c * W));
    std::vector<uint32_t> FA((size_t)r * k * N), FB((size_t)k * c * N), FC((size_t)r * c * N);
    for (int t = 0; t < np; ++t) {
        const NttPrime& P = g_primes[t];
        const uint32_t q = P.q;
        pool().run((int64_t)r * k + (int64_t)k * c, [&](int64_t idx) {
            const uint32_t* src;
            int64_t len;
            uint32_t* dst;
            if (idx < (int64_t)r * k) {
                src = A.a.data() + (size_t)idx * A.len;
                len = A.len;
                dst = FA.data() + (size_t)idx * N;
            } else {
                int64_t j = idx - (int64_t)r * k;
                src = B.a.data() + (size_t)j * B.len;
                len = B.len;
                dst = FB.data() + (size_t)j * N;
            }
            for (int64_t x = 0; x < len; ++x) dst[x] = src[x] >= q ? src[x] - q : src[x];
            std::memset(dst + len, 0, sizeof(uint32_t) * (N - (size_t)len));
            ntt_dif(dst, lg, P);
        });
        const uint32_t r32 = red64(P.mp, (uint64_t)1 << 32);
        const uint32_t ninv = invmod(P.mp, (uint32_t)(N % q));
        const size_t CH = 512;
        pool().run((int64_t)r * c, [&](int64_t idx) {
            int i = (int)(idx / c), l = (int)(idx % c);
            uint32_t* out = FC.data() + (size_t)idx * N;
            uint64_t lo32[CH], hi32[CH];
            for (size_t x0 = 0; x0 < N; x0 += CH) {
                const size_t cn = std::min(CH, N - x0);
                std::memset(lo32, 0, sizeof(uint64_t) * cn);
                std::memset(hi32, 0, sizeof(uint64_t) * cn);
                for (int j = 0; j < k; ++j) {
                    const uint32_t* a = FA.data() + ((size_t)i * k + j) * N + x0;
                    const uint32_t* b = FB.data() + ((size_t)j * c + l) * N + x0;
                    for (size_t x = 0; x < cn; ++x) {
                        uint64_t pr = (uint64_t)a[x] * b[x];
                        lo32[x] += pr & 0xffffffffu;
                        hi32[x] += pr >> 32;
                    }
                }
                for (size_t x = 0; x < cn; ++x)
                    out[x0 + x] = addmod(P.mp, red64(P.mp, lo32[x]), mulmod(P.mp, red64(P.mp, hi32[x]), r32));
            }
            ntt_dit_inv(out, lg, P);
            uint32_t* dst = res[t].data() + (size_t)idx * W;
            const uint32_t nip = shoup_pre(ninv, q);
            for (int64_t x = 0; x < W; ++x) dst[x] = mul_shoup(out[lo + x], ninv, nip, q);
        });
    }
    tables.unlock();
    // CRT (Garner) and reduction mod p
    C->resize(r, c, W);
    const size_t total = (size_t)r * c * W;
    if (np == 1) {
        for (size_t x = 0; x < total; ++x) C->a[x] = red64(mp, res[0][x]);
        return;
    }
    const NttPrime& P0 = g_primes[0];
    const NttPrime& P1 = g_primes[1];
    const NttPrime& P2 = g_primes[2];
    const uint32_t inv01 = invmod(P1.mp, P0.q % P1.q);                               // q0^-1 mod q1
    const uint32_t inv012 = invmod(P2.mp, mulmod(P2.mp, P0.q % P2.q, P1.q % P2.q));  // (q0 q1)^-1 mod q2
    const uint32_t q0p = red64(mp, P0.q), q01p = mulmod(mp, red64(mp, P0.q), red64(mp, P1.q));
    const int64_t chunks = (int64_t)((total + 65535) / 65536);
    pool().run(chunks, [&](int64_t ch) {
        size_t b = (size_t)ch * 65536, e = std::min(total, b + 65536);
        for (size_t x = b; x < e; ++x) {
            uint32_t a0 = res[0][x], a1 = res[1][x];
            // t1 = (a1 - a0) / q0 mod q1
            uint32_t d1 = a1 >= a0 % P1.q ? a1 - a0 % P1.q : a1 + P1.q - a0 % P1.q;
            uint32_t t1 = mulmod(P1.mp, d1, inv01);
            uint32_t v = addmod(mp, red64(mp, a0), mulmod(mp, q0p, red64(mp, t1)));
            if (np == 3) {
                uint32_t a2 = res[2][x];
                // x01 = a0 + q0 t1 mod q2 ; t2 = (a2 - x01) / (q0 q1) mod q2
                uint32_t x01 = (uint32_t)(((uint64_t)(a0 % P2.q) + mulmod(P2.mp, P0.q % P2.q, t1 % P2.q)) % P2.q);
                uint32_t d2 = a2 >= x01 ? a2 - x01 : a2 + P2.q - x01;
                uint32_t t2 = mulmod(P2.mp, d2, inv012);
                v = addmod(mp, v, mulmod(mp, q01p, red64(mp, t2)));
            }
            C->a[x] = v;
        }
    });
}

// ------------------------------------------------------------------ M-Basis (leaf)
namespace {

// sigma-basis of order sigma for G (m x n, G.len >= sigma), shifted degrees d in/out.
void mbasis(const PolyMat& G, int64_t sigma, std::vector<int64_t>& d, const ModP& mp, PolyMat* Pout) {
    const int m = G.rows, n = G.cols;
    // residual series Res = P G truncated at sigma, laid out [row][col][k]
    std::vector<uint32_t> res((size_t)m * n * sigma);
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < n; ++c) std::memcpy(&res[((size_t)r * n + c) * sigma], G.at(r, c), sizeof(uint32_t) * sigma);
    const int64_t plen = sigma + 1;
    std::vector<uint32_t> P((size_t)m * m * plen, 0);
    std::vector<int64_t> pdeg(m, 0);
    for (int r = 0; r < m; ++r) P[((size_t)r * m + r) * plen] = 1;
    auto R = [&](int r, int c) { return &res[((size_t)r * n + c) * sigma]; };
    auto PP = [&](int r, int c) { return &P[((size_t)r * m + c) * plen]; };
    std::vector<int> order(m);
    std::vector<std::pair<int, int>> piv;
    std::vector<uint32_t> pinv;
    for (int64_t k = 0; k < sigma; ++k) {
        for (int r = 0; r < m; ++r) order[r] = r;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
        piv.clear();
        pinv.clear();
        for (int i : order) {
            for (size_t t = 0; t < piv.size(); ++t) {
                int q = piv[t].first, c = piv[t].second;
                uint32_t v = R(i, c)[k];
                if (!v) continue;
                uint32_t f = mulmod(mp, v, pinv[t]);
                uint32_t nf = f ? mp.p - f : 0;
                for (int cc = 0; cc < n; ++cc) {
                    uint32_t* dst = R(i, cc);
                    const uint32_t* src = R(q, cc);
                    for (int64_t x = k; x < sigma; ++x)
                        if (src[x]) dst[x] = addmod(mp, dst[x], mulmod(mp, nf, src[x]));
                }
                for (int cc = 0; cc < m; ++cc) {
                    uint32_t* dst = PP(i, cc);
                    const uint32_t* src = PP(q, cc);
                    for (int64_t x = 0; x <= pdeg[q]; ++x)
                        if (src[x]) dst[x] = addmod(mp, dst[x], mulmod(mp, nf, src[x]));
                }
                pdeg[i] = std::max(pdeg[i], pdeg[q]);
            }
            int first = -1;
            for (int c = 0; c < n; ++c)
                if (R(i, c)[k]) {
                    first = c;
                    break;
                }
            if (first >= 0) {
                piv.emplace_back(i, first);
                pinv.push_back(invmod(mp, R(i, first)[k]));
            }
        }
        for (auto& pc : piv) {
            int q = pc.first;
            for (int cc = 0; cc < m; ++cc) {
                uint32_t* x = PP(q, cc);
                std::memmove(x + 1, x, sizeof(uint32_t) * (size_t)(pdeg[q] + 1));
                x[0] = 0;
            }
            pdeg[q] += 1;
            for (int cc = 0; cc < n; ++cc) {
                uint32_t* x = R(q, cc);
                if (sigma - k - 1 > 0) std::memmove(x + k + 1, x + k, sizeof(uint32_t) * (size_t)(sigma - k - 1));
                x[k] = 0;
            }
            d[q] += 1;
        }
    }
    int64_t maxdeg = 0;
    for (int r = 0; r < m; ++r) maxdeg = std::max(maxdeg, pdeg[r]);
    Pout->resize(m, m, maxdeg + 1);
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) std::memcpy(Pout->at(r, c), PP(r, c), sizeof(uint32_t) * (size_t)(maxdeg + 1));
}

int64_t g_leaf = 32;

void trim(PolyMat* P) {
    int64_t len = P->len;
    while (len > 1) {
        bool nz = false;
        for (int r = 0; r < P->rows && !nz; ++r)
            for (int c = 0; c < P->cols && !nz; ++c)
                if (P->at(r, c)[len - 1]) nz = true;
        if (nz) break;
        --len;
    }
    if (len == P->len) return;
    PolyMat Q;
    Q.resize(P->rows, P->cols, len);
    for (int r = 0; r < P->rows; ++r)
        for (int c = 0; c < P->cols; ++c) std::memcpy(Q.at(r, c), P->at(r, c), sizeof(uint32_t) * (size_t)len);
    *P = std::move(Q);
}

PolyMat truncate(const PolyMat& G, int64_t len) {
    PolyMat Q;
    Q.resize(G.rows, G.cols, len);
    for (int r = 0; r < G.rows; ++r)
        for (int c = 0; c < G.cols; ++c)
            std::memcpy(Q.at(r, c), G.at(r, c), sizeof(uint32_t) * (size_t)std::min(len, G.len));
    return Q;
}

void pmbasis(const PolyMat& G, int64_t sigma, std::vector<int64_t>& d, uint32_t p, PolyMat* P) {
    const ModP mp = ModP::make(p);
    if (sigma <= g_leaf) {
        mbasis(G, sigma, d, mp, P);
        return;
    }
    const int64_t s1 = sigma / 2, s2 = sigma - s1;
    PolyMat P1, P2, G2;
    pmbasis(G, s1, d, p, &P1);
    PolyMat Gt = truncate(G, sigma);
    polymat_mul(P1, Gt, s1, sigma, p, &G2);  // coefficients s1 .. sigma-1 of P1 G
    pmbasis(G2, s2, d, p, &P2);
    polymat_mul(P2, P1, 0, P1.len + P2.len - 1, p, P);
    trim(P);
}

Error build_G(const uint32_t* S, int64_t L, int32_t s, uint32_t p, PolyMat* G) {
    G->resize(2 * s, s, std::max<int64_t>(L, 1));
    for (int64_t k = 0; k < L; ++k)
        for (int i = 0; i < s; ++i)
            for (int j = 0; j < s; ++j) {
                uint32_t v = S[((size_t)k * s + i) * s + j];
                if (v >= p) return Error::inval("sequence entry not reduced mod p");
                G->at(i, j)[k] = v;
            }
    for (int i = 0; i < s; ++i) G->at(s + i, i)[0] = p - 1;  // -I
    return {};
}

Error extract(const PolyMat& P, const std::vector<int64_t>& d, int32_t s, Generator* out) {
    std::vector<int> rows(2 * s);
    for (int r = 0; r < 2 * s; ++r) rows[r] = r;
    std::stable_sort(rows.begin(), rows.end(), [&](int a, int b) { return d[a] < d[b]; });
    out->s = s;
    out->delta.assign(s, 0);
    int64_t maxd = 0;
    for (int i = 0; i < s; ++i) {
        out->delta[i] = d[rows[i]];
        maxd = std::max(maxd, d[rows[i]]);
    }
    out->P.resize(s, s, maxd + 1);
    for (int i = 0; i < s; ++i) {
        const int r = rows[i];
        for (int c = 0; c < s; ++c) {
            const uint32_t* src = P.at(r, c);
            for (int64_t x = 0; x < P.len; ++x) {
                if (!src[x]) continue;
                if (x > out->delta[i]) return {ESHORT_, "generator row degree exceeds its shifted degree"};
                out->P.at(i, c)[x] = src[x];
            }
        }
    }
    return {};
}

}  // namespace

Error min_generator(const uint32_t* S, int64_t L, int32_t s, uint32_t p, Generator* out, SigmaStats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    if (s < 1) return Error::inval("block size must be positive");
    PolyMat G, P;
    Error e = build_G(S, L, s, p, &G);
    if (!e.ok()) return e;
    std::vector<int64_t> d(2 * s, 0);
    for (int i = s; i < 2 * s; ++i) d[i] = 1;
    pmbasis(G, L, d, p, &P);
    e = extract(P, d, s, out);
    if (stats) {
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        stats->threads = sigma_threads();
    }
    return e;
}

Error min_generator_mbasis(const uint32_t* S, int64_t L, int32_t s, uint32_t p, Generator* out) {
    if (s < 1) return Error::inval("block size must be positive");
    PolyMat G, P;
    Error e = build_G(S, L, s, p, &G);
    if (!e.ok()) return e;
    std::vector<int64_t> d(2 * s, 0);
    for (int i = s; i < 2 * s; ++i) d[i] = 1;
    mbasis(G, L, d, ModP::make(p), &P);
    return extract(P, d, s, out);
}

Error check_generator(const Generator& g, const uint32_t* S, int64_t L, int64_t L_total, uint32_t p) {
    const ModP mp = ModP::make(p);
    const int s = g.s;
    const uint32_t r32 = red64(mp, (uint64_t)1 << 32);
    std::atomic<bool> bad{false};
    // coefficient c of p_i S, sum_j P_i[j] S[c - j], must vanish for max(L, delta_i) <= c < L_total.  Rows
    // run on the pool; per coefficient j the s x s term S[c - j] is read contiguously (columns b innermost),
    // and the 64-bit sums of low and high product halves stay exact (at most (delta_i + 1) s terms each).
    auto row = [&](int64_t i) {
        const int64_t di = g.delta[i];
        std::vector<uint64_t> lo(s), hi(s);
        std::vector<const uint32_t*> pa(s);
        for (int a = 0; a < s; ++a) pa[a] = g.P.at((int)i, a);
        for (int64_t c = std::max(L, di); c < L_total && !bad.load(std::memory_order_relaxed); ++c) {
            std::fill(lo.begin(), lo.end(), 0);
            std::fill(hi.begin(), hi.end(), 0);
            const int64_t jmax = std::min<int64_t>(std::min(di, c), g.P.len - 1);
            for (int64_t j = 0; j <= jmax; ++j) {
                const uint32_t* St = S + (size_t)(c - j) * s * s;
                for (int a = 0; a < s; ++a) {
                    const uint64_t w = pa[a][j];
                    if (!w) continue;
                    const uint32_t* srow = St + (size_t)a * s;
                    for (int b2 = 0; b2 < s; ++b2) {
                        const uint64_t pr = w * srow[b2];
                        lo[b2] += pr & 0xffffffffu;
                        hi[b2] += pr >> 32;
                    }
                }
            }
            for (int b2 = 0; b2 < s; ++b2)
                if (addmod(mp, red64(mp, lo[b2]), mulmod(mp, red64(mp, hi[b2]), r32))) bad.store(true);
        }
    };
    pool().run(s, row);
    if (bad.load()) return {ESHORT_, "generator fails on the check terms: the sequence is too short"};
    return {};
}

// ------------------------------------------------------------------ read-out
namespace {

// valuation of det M (s x s truncated power series, K coefficients); -1 if precision ran out
int64_t valuation_truncated(std::vector<std::vector<std::vector<uint32_t>>> A, int s, int64_t K, const ModP& mp) {
    auto val = [&](const std::vector<uint32_t>& v) {
        for (int64_t k = 0; k < K; ++k)
            if (v[k]) return k;
        return K;
    };
    int64_t total = 0;
    std::vector<uint32_t> q(K), uinv(K);
    for (int t = 0; t < s; ++t) {
        int64_t bv = K;
        int bi = -1, bj = -1;
        for (int i = t; i < s; ++i)
            for (int j = t; j < s; ++j) {
                int64_t v = val(A[i][j]);
                if (v < bv) {
                    bv = v;
                    bi = i;
                    bj = j;
                }
            }
        if (bi < 0) return -1;
        std::swap(A[t], A[bi]);
        for (int i = 0; i < s; ++i) std::swap(A[i][t], A[i][bj]);
        const int64_t v = bv, Kv = K - v;
        // inverse of the unit u = A[t][t] / x^v modulo x^(K - v)
        const std::vector<uint32_t>& piv = A[t][t];
        uint32_t inv0 = invmod(mp, piv[v]);
        for (int64_t k = 0; k < Kv; ++k) {
            uint32_t acc = k == 0 ? 1u : 0u;
            for (int64_t j = 1; j <= k; ++j)
                if (piv[v + j]) acc = addmod(mp, acc, mp.p - mulmod(mp, piv[v + j], uinv[k - j]));
            uinv[k] = mulmod(mp, acc, inv0);
        }
        for (int i = t + 1; i < s; ++i) {
            const std::vector<uint32_t>& w = A[i][t];
            std::fill(q.begin(), q.end(), 0u);
            for (int64_t a = 0; a < Kv; ++a)
                if (w[v + a])
                    for (int64_t b = 0; a + b < Kv; ++b) q[a + b] = addmod(mp, q[a + b], mulmod(mp, w[v + a], uinv[b]));
            for (int j = t; j < s; ++j) {
                const std::vector<uint32_t>& src = A[t][j];
                std::vector<uint32_t>& dst = A[i][j];
                for (int64_t a = 0; a < Kv; ++a)
                    if (q[a])
                        for (int64_t b = 0; a + b < K; ++b)
                            if (src[b]) dst[a + b] = addmod(mp, dst[a + b], mp.p - mulmod(mp, q[a], src[b]));
            }
        }
        total += v;
    }
    return total;
}

// valuation of det of the matrix whose (i, c) series is coef(i, c, k); -1 if det = 0
template <class Coef>
int64_t det_valuation(int s, int64_t bound, const ModP& mp, Coef coef) {
    int64_t K = 8;
    for (;;) {
        std::vector<std::vector<std::vector<uint32_t>>> A(s, std::vector<std::vector<uint32_t>>(s, std::vector<uint32_t>(K)));
        for (int i = 0; i < s; ++i)
            for (int c = 0; c < s; ++c)
                for (int64_t k = 0; k < K; ++k) A[i][c][k] = coef(i, c, k);
        int64_t v = valuation_truncated(std::move(A), s, K, mp);
        if (v >= 0) return v;
        if (K > bound) return -1;
        K *= 2;
    }
}

}  // namespace

Error rank_from_generator(const Generator& g, uint32_t p, int64_t* rank) {
    const ModP mp = ModP::make(p);
    const int s = g.s;
    int64_t sum_delta = 0;
    for (int64_t x : g.delta) sum_delta += x;
    const int64_t bound = sum_delta + 2;
    // val det P from the low coefficients of P
    int64_t vP = det_valuation(s, bound, mp, [&](int i, int c, int64_t k) -> uint32_t {
        return k < g.P.len ? g.P.at(i, c)[k] : 0u;
    });
    // val det F from the top coefficients of P (F_i(x) = x^delta_i P_i(1/x))
    int64_t vF = det_valuation(s, bound, mp, [&](int i, int c, int64_t k) -> uint32_t {
        int64_t j = g.delta[i] - k;
        return (j >= 0 && j < g.P.len) ? g.P.at(i, c)[j] : 0u;
    });
    if (vP < 0 || vF < 0) return {ESHORT_, "generator is singular"};
    *rank = sum_delta - vF - vP;
    return {};
}

}  // namespace bwr
