// Driver of the device sigma-basis: the PM-Basis recursion (Section 2.4) over
// device polynomial matrices.  Every size in the recursion is fixed by the
// order alone (a basis of order sigma has degree <= sigma), so the whole
// recursion is enqueued without waiting on the device; only the final
// shifted degrees and the chosen generator rows come back to the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <vector>

#include "sigma_gpu.h"

namespace bwr {

#define BWR_HIP(call)                                          \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return Error::device(e_, #call); \
    } while (0)

#define BWR_TRY(expr)              \
    do {                           \
        Error er_ = (expr);        \
        if (!er_.ok()) return er_; \
    } while (0)

namespace {

constexpr int MAX_LG = 20;

// Twiddle tables on the device, per device: [prime][value | shoup][2^MAX_LG]
struct DevTables {
    uint32_t* tw = nullptr;
    uint32_t* itw = nullptr;
    uint32_t q[3] = {0, 0, 0};
};

std::mutex g_tab_mu;
std::vector<DevTables> g_tabs;

Error device_tables(DevTables* out) {
    int dev = 0;
    BWR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_tab_mu);
    if ((int)g_tabs.size() <= dev) g_tabs.resize(dev + 1);
    DevTables& T = g_tabs[dev];
    if (!T.tw) {
        const size_t N = (size_t)1 << MAX_LG;
        std::vector<uint32_t> h_tw(3 * 2 * N), h_itw(3 * 2 * N);
        for (int t = 0; t < 3; ++t)
            ntt_tables(t, MAX_LG, &T.q[t], &h_tw[(2 * t) * N], &h_tw[(2 * t + 1) * N], &h_itw[(2 * t) * N],
                       &h_itw[(2 * t + 1) * N]);
        // uploaded on a private non-blocking stream: an operation on the legacy stream would synchronize with
        // every blocking stream, and fails while one of them is being captured into a graph by another thread
        uint32_t *a = nullptr, *b = nullptr;
        hipStream_t up = nullptr;
        BWR_HIP(hipStreamCreateWithFlags(&up, hipStreamNonBlocking));
        hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&a), h_tw.size() * 4, up);
        if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&b), h_itw.size() * 4, up);
        if (e == hipSuccess) e = hipMemcpyAsync(a, h_tw.data(), h_tw.size() * 4, hipMemcpyHostToDevice, up);
        if (e == hipSuccess) e = hipMemcpyAsync(b, h_itw.data(), h_itw.size() * 4, hipMemcpyHostToDevice, up);
        const hipError_t es = hipStreamSynchronize(up);  // the host tables are read before they go out of scope
        (void)hipStreamDestroy(up);
        if (e == hipSuccess) e = es;
        if (e != hipSuccess) return Error::device(e, "sigma-basis transform tables");
        T.tw = a;
        T.itw = b;
    }
    *out = T;
    return {};
}

uint32_t shoup(uint32_t w, uint32_t q) { return (uint32_t)(((uint64_t)w << 32) / q); }

NttConsts make_consts(const DevTables& T, int lg, const PrimeBatch& pb) {
    NttConsts c{};
    for (int t = 0; t < 3; ++t) {
        c.q[t] = T.q[t];
        c.mq[t] = ModP::make(T.q[t]);
        c.r32[t] = red64(c.mq[t], (uint64_t)1 << 32);
        c.ninv[t] = invmod(c.mq[t], (uint32_t)(((uint64_t)1 << lg) % T.q[t]));
        c.ninvp[t] = shoup(c.ninv[t], T.q[t]);
    }
    c.inv01 = invmod(c.mq[1], T.q[0] % T.q[1]);
    c.inv012 = invmod(c.mq[2], mulmod(c.mq[2], T.q[0] % T.q[2], T.q[1] % T.q[2]));
    for (int b = 0; b < pb.n; ++b) {
        const ModP& mp = pb.mp[b];
        c.q0p[b] = red64(mp, T.q[0]);
        c.q01p[b] = mulmod(mp, red64(mp, T.q[0]), red64(mp, T.q[1]));
    }
    c.tw_stride = (int64_t)1 << MAX_LG;
    return c;
}

int ceil_log2(int64_t x) {
    int l = 0;
    while (((int64_t)1 << l) < x) ++l;
    return l;
}

Error alloc_poly(int rows, int cols, int64_t len, int batch, hipStream_t st, DevBuf* buf, DPoly* P) {
    BWR_TRY(buf->alloc(sizeof(uint32_t) * (size_t)batch * rows * cols * (size_t)std::max<int64_t>(len, 1), st));
    P->rows = rows;
    P->cols = cols;
    P->len = len;
    P->ld = len;
    P->ptr = buf->as<uint32_t>();
    P->batch = batch;
    return {};
}

PrimeBatch make_batch(const uint32_t* p, int nb) {
    PrimeBatch pb;
    pb.n = nb;
    for (int b = 0; b < nb; ++b) pb.mp[b] = ModP::make(p[b]);
    return pb;
}

}  // namespace

int gpu_leaf_order(int s) {
    const int m = 2 * s, n = s;
    if (s >= 1 && s <= LEAF2_MAX_S) {
        // LDS per workgroup of this device, less what the kernel declares statically
        int dev = 0, lds = 64 * 1024;
        if (hipGetDevice(&dev) == hipSuccess) {
            int v = 0;
            if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
                lds = std::min(v, 160 * 1024);
        }
        const size_t budget = (size_t)lds - 8 * 1024;
        for (int sg = 32; sg >= 1; sg >>= 1)
            if (mbasis_leaf2_lds(m, n, sg) <= budget) return sg;
        return 0;
    }
    for (int sg = 32; sg >= 1; sg >>= 1)
        if (mbasis_leaf_lds(m, n, sg) <= 60 * 1024 && m <= 128) return sg;
    return 0;
}

Error gpu_polymat_mul(const DPoly& A, const DPoly& B, int64_t lo, int64_t hi, const PrimeBatch& pb, DPoly* C,
                      DevBuf* Cbuf, hipStream_t st) {
    const int r = A.rows, k = A.cols, c = B.cols, nbt = A.batch;
    if (A.cols != B.rows || A.batch != B.batch || A.batch != pb.n || pb.n < 1 || pb.n > SIGMA_BATCH_MAX)
        return Error::inval("polynomial matrix product: shapes or batch do not match");
    const int64_t W = hi - lo;
    BWR_TRY(alloc_poly(r, c, W, nbt, st, Cbuf, C));
    const int64_t minlen = std::min(A.len, B.len);
    if (minlen <= 32) {
        if (A.ld != A.len || B.ld != B.len) {
            // compact copies so the schoolbook kernel can assume dense rows
            DevBuf ab, bb;
            DPoly Ac, Bc;
            BWR_TRY(alloc_poly(A.rows, A.cols, A.len, nbt, st, &ab, &Ac));
            BWR_TRY(alloc_poly(B.rows, B.cols, B.len, nbt, st, &bb, &Bc));
            BWR_HIP(gpu_copy_rows(Ac.ptr, A.len, A.ptr, A.ld, A.len, (int64_t)nbt * A.rows * A.cols, st));
            BWR_HIP(gpu_copy_rows(Bc.ptr, B.len, B.ptr, B.ld, B.len, (int64_t)nbt * B.rows * B.cols, st));
            BWR_HIP(gpu_schoolbook(Ac.ptr, A.len, Bc.ptr, B.len, r, k, c, lo, W, pb, C->ptr, st));
            return {};
        }
        BWR_HIP(gpu_schoolbook(A.ptr, A.len, B.ptr, B.len, r, k, c, lo, W, pb, C->ptr, st));
        return {};
    }
    DevTables T;
    BWR_TRY(device_tables(&T));
    const uint32_t p = pb.max_p();
    const double bound = (double)k * (double)minlen * (double)(p - 1) * (double)(p - 1);
    int np = 1;
    double prod = (double)T.q[0];
    while (prod <= bound * 1.0001 && np < 3) prod *= (double)T.q[np++];
    if (prod <= bound) return Error::inval("polynomial product exceeds the CRT range");
    const int lg = ceil_log2(std::max<int64_t>(hi, A.len + B.len - 1 - lo));
    if (lg > MAX_LG) return Error::inval("polynomial product too long for the transform tables");
    const int64_t N = (int64_t)1 << lg;
    const NttConsts cs = make_consts(T, lg, pb);
    DevBuf fa, fb, fc;
    const int na = nbt * r * k, nbb = nbt * k * c, nc = nbt * r * c;
    BWR_TRY(fa.alloc(sizeof(uint32_t) * (size_t)np * na * N, st));
    BWR_TRY(fb.alloc(sizeof(uint32_t) * (size_t)np * nbb * N, st));
    BWR_TRY(fc.alloc(sizeof(uint32_t) * (size_t)np * nc * N, st));
    BWR_HIP(gpu_load_polys(A.ptr, A.ld, A.len, 0, na, N, np, cs, fa.as<uint32_t>(), st));
    BWR_HIP(gpu_load_polys(B.ptr, B.ld, B.len, 0, nbb, N, np, cs, fb.as<uint32_t>(), st));
    BWR_HIP(gpu_ntt(fa.as<uint32_t>(), lg, na, np, cs, T.tw, T.itw, true, st));
    BWR_HIP(gpu_ntt(fb.as<uint32_t>(), lg, nbb, np, cs, T.tw, T.itw, true, st));
    BWR_HIP(gpu_pointwise(fa.as<uint32_t>(), fb.as<uint32_t>(), fc.as<uint32_t>(), r, k, c, nbt, N, np, cs, st));
    BWR_HIP(gpu_ntt(fc.as<uint32_t>(), lg, nc, np, cs, T.tw, T.itw, false, st));
    BWR_HIP(gpu_crt(fc.as<uint32_t>(), nc, r * c, N, lo, W, np, cs, pb, C->ptr, st));
    return {};
}

namespace {

struct Recur {
    PrimeBatch pb;
    int m, n, leaf;
    int64_t* d;  // device shifted degrees, m per batch element
    hipStream_t st;
};

// P (m x m, len sigma + 1) = order-sigma basis of G (m x n, coefficients 0 .. sigma - 1, stride G.ld), for
// every batch element
Error pm(const Recur& R, const DPoly& G, int64_t sigma, DPoly* P, DevBuf* Pbuf) {
    if (sigma <= R.leaf) {
        BWR_TRY(alloc_poly(R.m, R.m, sigma + 1, G.batch, R.st, Pbuf, P));
        BWR_HIP(gpu_mbasis_leaf(G.ptr, G.ld, (int64_t)G.rows * G.cols * G.ld, R.m, R.n, (int)sigma, R.d, P->ptr, P->ld,
                                (int64_t)P->rows * P->cols * P->ld, R.pb, R.st));
        return {};
    }
    const int64_t s1 = sigma / 2, s2 = sigma - s1;
    DevBuf b1, bg2, b2;
    DPoly P1, G2, P2;
    BWR_TRY(pm(R, G, s1, &P1, &b1));
    DPoly Gs = G;
    Gs.len = sigma;
    BWR_TRY(gpu_polymat_mul(P1, Gs, s1, sigma, R.pb, &G2, &bg2, R.st));
    BWR_TRY(pm(R, G2, s2, &P2, &b2));
    BWR_TRY(gpu_polymat_mul(P2, P1, 0, sigma + 1, R.pb, P, Pbuf, R.st));
    return {};
}

}  // namespace

Error OnlineGenerator::begin(const uint32_t* const* S_dev, int nb, int64_t L, int32_t s, const uint32_t* p,
                             int64_t min_chunk, hipStream_t st) {
    leaf_ = gpu_leaf_order(s);
    if (!leaf_) return Error::inval("block size too large for the device sigma-basis");
    if (s > 64) return Error::inval("block size too large for the device sigma-basis");
    if (nb < 1 || nb > SIGMA_BATCH_MAX) return Error::inval("sigma-basis batch must hold 1 to 4 sequences");
    pb_ = make_batch(p, nb);
    if (!pb_.small() && !pb_.large()) return Error::inval("a sigma-basis batch mixes 16-bit and larger primes");
    for (int b = 0; b < nb; ++b) S_[b] = S_dev[b];
    L_ = L;
    s_ = s;
    st_ = st;
    built_ = done_ = 0;
    next_ = pending_ = 0;
    early_ = false;
    ecs_ = EarlyCutState{};
    conv_.store(0);
    cuts_.clear();
    if (L > 0) {
        int64_t c = 0;
        if (min_chunk > 0) {
            // quarters while at least half of the range is left, then halves of the rest: early chunks
            // start while most of the sequence is still to come, the last ones leave a short tail
            while ((L - c) / 2 >= min_chunk) {
                c += std::max<int64_t>(std::min<int64_t>(L / 4, (L - c) / 2), 1);
                cuts_.push_back(c);
            }
        }
        cuts_.push_back(L);
    }
    const int m = 2 * s, n = s;
    // G_b = [S_b; -I] as m x n device polynomial matrices, filled as the terms arrive
    BWR_TRY(alloc_poly(m, n, std::max<int64_t>(L, 1), nb, st, &gb_, &G_));
    std::vector<int64_t> d0((size_t)nb * m, 0);
    for (int b = 0; b < nb; ++b)
        for (int i = s; i < m; ++i) d0[(size_t)b * m + i] = 1;
    BWR_TRY(db_.alloc(sizeof(int64_t) * d0.size(), st));
    BWR_HIP(hipMemcpyAsync(db_.as<void>(), d0.data(), sizeof(int64_t) * d0.size(), hipMemcpyHostToDevice, st));
    BWR_HIP(hipStreamSynchronize(st));  // the host buffer above must outlive its copy
    return {};
}

Error OnlineGenerator::begin_early(const uint32_t* S_dev, int64_t L, int32_t s, uint32_t p, int64_t step,
                                   int64_t verify, hipStream_t st) {
    if (step < 1 || verify < 1) return Error::inval("early termination needs positive chunk lengths");
    BWR_TRY(begin(&S_dev, 1, L, s, &p, 0, st));
    early_ = true;
    step_ = step;
    verify_ = verify;
    force_at_ = 0;
    ecs_ = EarlyCutState{};
    ecs_.vstep = verify;
    cuts_.clear();
    if (L > 0) cuts_.push_back(std::min(L, std::max(step, L / 8)));
    return {};
}

// After the chunk ending at done_ (worker thread): the generator rows' degree sum against the previous cut's
// decides convergence and the next cut (early_cut.h).
Error OnlineGenerator::after_chunk_early() {
    std::vector<int64_t> d(2 * s_);
    BWR_HIP(hipMemcpyAsync(d.data(), db_.as<void>(), sizeof(int64_t) * d.size(), hipMemcpyDeviceToHost, st_));
    BWR_HIP(hipStreamSynchronize(st_));
    const EarlyCutDecision dec = early_cut_after_chunk(d.data(), s_, done_, L_, step_, verify_, &ecs_);
    if (dec.converged || (force_at_ > 0 && done_ >= force_at_)) {
        conv_.store(done_);
        return {};
    }
    if (dec.next_cut >= 0) cuts_.push_back(dec.next_cut);
    return {};
}

OnlineGenerator::~OnlineGenerator() { (void)join_worker(); }

void OnlineGenerator::feed_async(int64_t avail, hipEvent_t ready) {
    // in early-termination mode the worker owns the cuts (next_boundary() is not used there)
    if (!early_)
        while (pending_ < (int)cuts_.size() && cuts_[pending_] <= avail) ++pending_;
    {
        std::lock_guard<std::mutex> lk(mu_);
        queue_.emplace_back(avail, ready);
    }
    if (!worker_.joinable()) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        worker_ = std::thread([this, dev] {
            (void)hipSetDevice(dev);
            for (;;) {
                std::pair<int64_t, hipEvent_t> item;
                {
                    std::unique_lock<std::mutex> lk(mu_);
                    cv_.wait(lk, [&] { return closing_ || !queue_.empty(); });
                    if (queue_.empty()) return;
                    item = queue_.front();
                    queue_.pop_front();
                }
                Error e = werr_.ok() ? feed(item.first, item.second) : Error{};
                if (item.second) (void)hipEventDestroy(item.second);  // the wait above is already enqueued
                if (!e.ok()) {
                    std::lock_guard<std::mutex> lk(mu_);
                    werr_ = e;
                }
            }
        });
    }
    cv_.notify_one();
}

Error OnlineGenerator::join_worker() {
    if (worker_.joinable()) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            closing_ = true;
        }
        cv_.notify_one();
        worker_.join();
    }
    for (auto& it : queue_)
        if (it.second) (void)hipEventDestroy(it.second);
    queue_.clear();
    return werr_;
}

Error OnlineGenerator::feed(int64_t avail, hipEvent_t ready) {
    avail = std::min(avail, L_);
    if (avail <= built_ || conv_.load() > 0) return {};
    // a host wait (feed_async runs this on the generator's own thread): a stream wait on an event of the
    // producer's stream would join a graph capture that stream may have begun since the event was recorded
    if (ready) BWR_HIP(hipEventSynchronize(ready));
    const int64_t gbs = (int64_t)G_.rows * G_.cols * G_.ld;
    for (int b = 0; b < pb_.n; ++b)
        BWR_HIP(gpu_build_G(S_[b], L_, s_, pb_.mp[b].p, G_.ptr + b * gbs, G_.ld, built_, avail, st_));
    built_ = avail;
    const Recur R{pb_, 2 * s_, s_, leaf_, db_.as<int64_t>(), st_};
    while (next_ < (int)cuts_.size() && cuts_[next_] <= built_) {
        const int64_t c0 = done_, c1 = cuts_[next_];
        DPoly Gs = G_;
        Gs.len = c1;
        if (c0 == 0) {
            BWR_TRY(pm(R, Gs, c1, &Q_, &qb_));
        } else {
            DevBuf rb, pb, nb;
            DPoly Rc, P, Qn;
            BWR_TRY(gpu_polymat_mul(Q_, Gs, c0, c1, pb_, &Rc, &rb, st_));
            BWR_TRY(pm(R, Rc, c1 - c0, &P, &pb));
            BWR_TRY(gpu_polymat_mul(P, Q_, 0, c1 + 1, pb_, &Qn, &nb, st_));
            qb_ = std::move(nb);
            Q_ = Qn;
        }
        done_ = c1;
        ++next_;
        if (early_) {
            BWR_TRY(after_chunk_early());
            if (conv_.load() > 0) break;
        }
    }
    return {};
}



Error OnlineGenerator::finish(Generator* out) {
    BWR_TRY(join_worker());
    if (done_ != L_ && !(conv_.load() > 0 && done_ == conv_.load()))
        return Error::inval("sigma-basis finished before every term was fed");
    const int m = 2 * s_, s = s_, nbt = pb_.n;
    DevBuf ib;
    DPoly P = Q_;
    if (L_ == 0) {  // the basis of order 0 is the identity
        BWR_TRY(alloc_poly(m, m, 1, nbt, st_, &ib, &P));
        std::vector<uint32_t> I((size_t)nbt * m * m, 0);
        for (int b = 0; b < nbt; ++b)
            for (int i = 0; i < m; ++i) I[((size_t)b * m + i) * m + i] = 1;
        BWR_HIP(hipMemcpyAsync(P.ptr, I.data(), 4 * I.size(), hipMemcpyHostToDevice, st_));
        BWR_HIP(hipStreamSynchronize(st_));
    }
    std::vector<int64_t> d((size_t)nbt * m);
    BWR_HIP(hipMemcpyAsync(d.data(), db_.as<void>(), sizeof(int64_t) * d.size(), hipMemcpyDeviceToHost, st_));
    BWR_HIP(hipStreamSynchronize(st_));
    // per batch element: the s rows of smallest shifted degree (ties: row index), gathered on the device
    // (coefficients above each degree zeroed and checked), then one copy each
    std::vector<DevBuf> obs(nbt);
    DevBuf fb;
    BWR_TRY(fb.alloc(sizeof(int32_t) * nbt, st_));
    BWR_HIP(hipMemsetAsync(fb.as<void>(), 0, sizeof(int32_t) * nbt, st_));
    const int64_t pbs = (int64_t)P.rows * P.cols * P.ld;
    for (int b = 0; b < nbt; ++b) {
        const int64_t* db = d.data() + (size_t)b * m;
        std::vector<int> rows(m);
        for (int r = 0; r < m; ++r) rows[r] = r;
        std::stable_sort(rows.begin(), rows.end(), [&](int a, int c) { return db[a] < db[c]; });
        Generator& g = out[b];
        g.s = s;
        g.delta.assign(s, 0);
        int64_t maxd = 0;
        for (int i = 0; i < s; ++i) {
            g.delta[i] = db[rows[i]];
            maxd = std::max(maxd, g.delta[i]);
        }
        g.P.resize(s, s, maxd + 1);
        GenRows gr{};
        for (int i = 0; i < s; ++i) {
            gr.row[i] = rows[i];
            gr.delta[i] = g.delta[i];
        }
        BWR_TRY(obs[b].alloc(sizeof(uint32_t) * g.P.a.size(), st_));
        BWR_HIP(gpu_extract_rows(P.ptr + b * pbs, P.ld, P.len, m, s, gr, maxd + 1, obs[b].as<uint32_t>(),
                                 fb.as<int32_t>() + b, st_));
        BWR_HIP(hipMemcpyAsync(g.P.a.data(), obs[b].as<void>(), sizeof(uint32_t) * g.P.a.size(),
                               hipMemcpyDeviceToHost, st_));
    }
    std::vector<int32_t> bad(nbt, 0);
    BWR_HIP(hipMemcpyAsync(bad.data(), fb.as<void>(), sizeof(int32_t) * nbt, hipMemcpyDeviceToHost, st_));
    BWR_HIP(hipStreamSynchronize(st_));
    for (int b = 0; b < nbt; ++b)
        if (bad[b]) return {ESHORT_, "generator row degree exceeds its shifted degree"};
    return {};
}

Error gpu_min_generator(const uint32_t* S_dev, int64_t L, int32_t s, uint32_t p, hipStream_t st, Generator* out,
                        SigmaStats* stats, int64_t min_chunk) {
    auto t0 = std::chrono::steady_clock::now();
    OnlineGenerator og;
    BWR_TRY(og.begin(&S_dev, 1, L, s, &p, min_chunk, st));
    BWR_TRY(og.feed(L, nullptr));
    BWR_TRY(og.finish(out));
    if (stats) {
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        stats->threads = 0;
    }
    return {};
}

Error gpu_min_generators(const uint32_t* const* S_dev, int nb, int64_t L, int32_t s, const uint32_t* p,
                         hipStream_t st, Generator* out) {
    OnlineGenerator og;
    BWR_TRY(og.begin(S_dev, nb, L, s, p, 0, st));
    BWR_TRY(og.feed(L, nullptr));
    return og.finish(out);
}

}  // namespace bwr
