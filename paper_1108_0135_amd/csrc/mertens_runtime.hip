// Host runtime and C ABI of the gfx950 Mertens library (see include/mertens.h).
//
// The runtime plans a sweep (Section 2 blocking: u, L per query, sieve limit,
// sieving primes), owns every device buffer, and issues the per-block kernel
// sequence of Section 3 on one HIP stream:
//   block setup -> sieve -> segment scan -> fixup -> update prep -> item scan
//   -> persistent update
// followed by finalize and collect.  No host synchronisation happens inside
// the sweep; the host only waits for the final results.
#include "mertens.h"
#include "mertens_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace mrt;

namespace {

std::string g_last_error = "no error";

void set_error(const char *what, hipError_t e, const char *file, int line)
{
    char buf[512];
    snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    g_last_error = buf;
}

void set_error_text(const char *text) { g_last_error = text; }

#define HIPCHK(expr)                                         \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) {                              \
            set_error(#expr, e_, __FILE__, __LINE__);        \
            return MERTENS_EIO;                              \
        }                                                    \
    } while (0)

#define RCCHK(expr)              \
    do {                         \
        int rc_ = (expr);        \
        if (rc_ != 0)            \
            return rc_;          \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    template <class T>
    T *as() const { return static_cast<T *>(p); }
    void release()
    {
        if (p)
            (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

int ensure(DevBuf &b, size_t bytes)
{
    if (bytes < 64)
        bytes = 64;
    if (b.bytes >= bytes)
        return 0;
    b.release();
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        set_error("hipMalloc", e, __FILE__, __LINE__);
        (void)hipGetLastError();
        return MERTENS_ENOMEM;
    }
    b.bytes = bytes;
    return 0;
}

uint64_t isqrt_host(uint64_t v)
{
    uint64_t r = (uint64_t)std::sqrt((double)v);
    while (r > 0xFFFFFFFFull || r * r > v)
        r--;
    while (r < 0xFFFFFFFFull && (r + 1) * (r + 1) <= v)
        r++;
    return r;
}

uint64_t ceil_sqrt_host(uint64_t v)
{
    uint64_t r = isqrt_host(v);
    return (r * r < v) ? r + 1 : r;
}

uint8_t log_prime_host(uint64_t p)
{
    uint32_t l = 0;
    while ((1ull << l) < p)
        l++;
    return (uint8_t)(l | 1u);  // ceil(log2 p) | 1
}

struct Ctx {
    bool ready = false;
    int device = 0;
    int ncu = 256;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    uint64_t u_req = 0, block_req = 0;
    // tuning
    double beta = 0.2;
    uint32_t ychunk = 4096, kchunk = 2048, klchunk = 256, waves_per_cu = 16;
    // sieving primes (>= 5) up to psieve, and the pre-sieved pattern
    uint64_t psieve = 0;
    std::vector<uint32_t> h_primes;
    DevBuf pres, res2, pattern;
    // block buffers
    DevBuf masks, mb, seg_sum, seg_off, carry;
    // query buffers
    DevBuf q_n, q_L, q_g0, x_m, x_Y, x_K, x_k0, S, A, x_klo, x_khi;
    DevBuf tile_q, tile_x0, tile_nx, tile_g0, tile_ymax, tile_klo, tile_khi, tile_mode, tile_nmu,
        tile_items, counter, pair_stats, out_dev;
    // last query (for byproducts): per caller index, L and first global index
    std::vector<uint64_t> last_L, last_g0;
    bool last_valid = false;
    double stats[16] = {0};
    std::vector<hipEvent_t> events;
};

Ctx g;

void free_all()
{
    DevBuf *bufs[] = {&g.pres, &g.res2, &g.pattern, &g.masks, &g.mb,
                      &g.seg_sum, &g.seg_off, &g.carry, &g.q_n, &g.q_L, &g.q_g0, &g.x_m,
                      &g.x_Y, &g.x_K, &g.x_k0, &g.S, &g.A, &g.x_klo, &g.x_khi, &g.tile_q,
                      &g.tile_x0, &g.tile_nx, &g.tile_g0, &g.tile_ymax, &g.tile_klo,
                      &g.tile_khi, &g.tile_mode, &g.tile_nmu, &g.tile_items, &g.counter,
                      &g.pair_stats, &g.out_dev};
    for (DevBuf *b : bufs)
        b->release();
    for (hipEvent_t e : g.events)
        (void)hipEventDestroy(e);
    g.events.clear();
    if (g.own_stream)
        (void)hipStreamDestroy(g.own_stream);
    g.own_stream = nullptr;
    g.stream = nullptr;
    g.h_primes.clear();
    g.psieve = 0;
    g.last_L.clear();
    g.last_g0.clear();
    g.last_valid = false;
    g.ready = false;
}

// Sieving primes p in [5, limit] (plain Eratosthenes on odd numbers) and
// their device copy as {p, residue} pairs.  Grows only.
int ensure_primes(uint64_t limit)
{
    if (limit <= g.psieve)
        return 0;
    std::vector<uint8_t> comp(limit / 2 + 1, 0);  // comp[i] <=> 2i+1 composite
    for (uint64_t i = 3; i * i <= limit; i += 2)
        if (!comp[i / 2])
            for (uint64_t j = i * i; j <= limit; j += 2 * i)
                comp[j / 2] = 1;
    std::vector<uint32_t> pr, pairs;
    for (uint64_t v = 5; v <= limit; v += 2)
        if (!comp[v / 2]) {
            pr.push_back((uint32_t)v);
            pairs.push_back((uint32_t)v);
            pairs.push_back(0u);
        }
    const size_t np = pr.size();
    RCCHK(ensure(g.pres, np * 8));
    RCCHK(ensure(g.res2, np * 8));
    HIPCHK(hipMemcpy(g.pres.p, pairs.data(), np * 8, hipMemcpyHostToDevice));
    g.h_primes.swap(pr);
    g.psieve = limit;
    return 0;
}

// Pattern of the modified sieve for the primes 2, 3, 5, 7, 11, 13 and the
// squares 4, 9 (period 180180), extended by one segment so a segment's
// initial state is one straight copy.
int upload_pattern()
{
    const uint32_t small[6] = {2, 3, 5, 7, 11, 13};
    std::vector<uint8_t> pat((size_t)PAT_WORDS * 4, 0);
    for (size_t i = 0; i < pat.size(); ++i) {
        const uint32_t r = (uint32_t)(i % PAT);
        uint32_t a = 0;
        for (uint32_t p : small)
            if (r % p == 0)
                a += log_prime_host(p);
        if (r % 4 == 0 || r % 9 == 0)
            a |= 0x80u;
        pat[i] = (uint8_t)a;
    }
    RCCHK(ensure(g.pattern, pat.size()));
    HIPCHK(hipMemcpy(g.pattern.p, pat.data(), pat.size(), hipMemcpyHostToDevice));
    return 0;
}

uint32_t count_primes_upto(uint64_t v)  // # table primes p <= v
{
    return (uint32_t)(std::upper_bound(g.h_primes.begin(), g.h_primes.end(),
                                       (uint64_t)v,
                                       [](uint64_t a, uint32_t b) { return a < b; }) -
                      g.h_primes.begin());
}

uint32_t count_squares_upto(uint64_t v)  // # table primes with p^2 <= v
{
    return count_primes_upto(isqrt_host(v));
}

int ensure_block_buffers(uint64_t B)
{
    const uint64_t words = B / 64;
    const uint64_t nseg = B / SEG;
    RCCHK(ensure(g.masks, words * 16));
    RCCHK(ensure(g.mb, words * 8));
    RCCHK(ensure(g.seg_sum, nseg * 4));
    RCCHK(ensure(g.seg_off, nseg * 8));
    RCCHK(ensure(g.carry, 64));
    return 0;
}

BlockArgs make_block(uint64_t y1, uint64_t y2)
{
    BlockArgs b;
    b.y1 = y1;
    b.y2 = y2;
    b.nseg = (uint32_t)((y2 - y1) / SEG + 1);
    b.n_small = count_primes_upto(SMALL_P - 1);
    b.n_sieve = (uint32_t)g.h_primes.size();
    b.n_sq = count_squares_upto(y2);
    b.n_sq_lds = std::min(count_primes_upto(SQ_LDS_P), b.n_sq);
    b.pat_off = (uint32_t)(y1 % PAT);
    b.pres = g.pres.as<uint2>();
    b.res2 = g.res2.as<uint64_t>();
    b.pat32 = g.pattern.as<uint32_t>();
    b.masks = g.masks.as<uint64_t>();
    b.mb = g.mb.as<int64_t>();
    b.seg_sum = g.seg_sum.as<int32_t>();
    b.seg_off = g.seg_off.as<int64_t>();
    b.carry = g.carry.as<int64_t>();
    return b;
}

// Sieve one block: residue setup, then the sieve kernel (an event may be
// recorded between the two so the sieve kernel is timed alone).
int sieve_block(const BlockArgs &b, hipEvent_t between = nullptr)
{
    HIPCHK(launch_block_setup(b, g.stream));
    if (between)
        HIPCHK(hipEventRecord(between, g.stream));
    HIPCHK(launch_sieve(b, g.stream));
    HIPCHK(launch_square_fix(b, g.stream));
    return 0;
}

int scan_block(const BlockArgs &b)
{
    HIPCHK(launch_scan_words(b, g.stream));
    HIPCHK(launch_scan_segments(b, g.stream));
    HIPCHK(launch_fixup(b, g.stream));
    return 0;
}

hipEvent_t event_at(size_t i)
{
    while (g.events.size() <= i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess)
            return nullptr;
        g.events.push_back(e);
    }
    return g.events[i];
}

float elapsed(size_t a, size_t b)
{
    float ms = 0;
    if (hipEventElapsedTime(&ms, g.events[a], g.events[b]) != hipSuccess)
        return 0;
    return ms;
}

uint64_t choose_block(uint64_t ymax)
{
    if (g.block_req)
        return g.block_req;
    uint64_t need = (ymax / SEG + 1) * SEG;
    return std::min<uint64_t>(need, 1ull << 30);
}

// The sweep for nonzero arguments ns[]: fills A on the device and the
// results into res[] (host).
int run_query(const std::vector<uint64_t> &ns, std::vector<int64_t> &res,
              std::vector<uint64_t> &Ls, std::vector<uint64_t> &g0s)
{
    const size_t nq = ns.size();
    // ---- plan (a0): u, L, sieve limit
    uint64_t u = g.u_req;
    if (u == 0) {
        long double sum = 0;
        for (uint64_t n : ns)
            sum += (long double)n;
        u = (uint64_t)std::ceil(std::pow((double)sum, 2.0 / 3.0));
        if (u < 2)
            u = 2;
    }
    Ls.resize(nq);
    g0s.resize(nq);
    uint64_t X = 0, ymax = 0;
    for (size_t i = 0; i < nq; ++i) {
        uint64_t L = ns[i] / u;
        if (L < 1)
            L = 1;
        if (L >= (1ull << 31)) {
            set_error_text("u too small: some n would need an array of 2^31 or more entries");
            return MERTENS_EINVAL;
        }
        Ls[i] = L;
        g0s[i] = X;
        X += L;
        ymax = std::max<uint64_t>(ymax, ns[i] / (L + 1));
    }
    // tiles of 64 consecutive x per query
    std::vector<uint32_t> t_q, t_x0, t_nx;
    std::vector<uint64_t> t_g0;
    for (size_t i = 0; i < nq; ++i)
        for (uint64_t x0 = 1; x0 <= Ls[i]; x0 += TILE) {
            t_q.push_back((uint32_t)i);
            t_x0.push_back((uint32_t)x0);
            t_nx.push_back((uint32_t)std::min<uint64_t>(TILE, Ls[i] - x0 + 1));
            t_g0.push_back(g0s[i] + x0 - 1);
        }
    const size_t nt = t_q.size();
    if (nt >= (1ull << 31)) {
        set_error_text("too many tiles");
        return MERTENS_EINVAL;
    }

    const uint64_t psieve = std::max<uint64_t>(ceil_sqrt_host(ymax), 1024);
    RCCHK(ensure_primes(psieve));
    const uint64_t B = choose_block(ymax);
    RCCHK(ensure_block_buffers(B));

    RCCHK(ensure(g.q_n, nq * 8));
    RCCHK(ensure(g.q_L, nq * 8));
    RCCHK(ensure(g.q_g0, nq * 8));
    DevBuf *xb[] = {&g.x_m, &g.x_Y, &g.x_K, &g.x_k0, &g.S, &g.A, &g.x_klo, &g.x_khi};
    for (DevBuf *b : xb)
        RCCHK(ensure(*b, X * 8));
    RCCHK(ensure(g.tile_q, nt * 4));
    RCCHK(ensure(g.tile_x0, nt * 4));
    RCCHK(ensure(g.tile_nx, nt * 4));
    RCCHK(ensure(g.tile_mode, nt * 4));
    RCCHK(ensure(g.tile_nmu, nt * 4));
    RCCHK(ensure(g.tile_g0, nt * 8));
    RCCHK(ensure(g.tile_ymax, nt * 8));
    RCCHK(ensure(g.tile_klo, nt * 8));
    RCCHK(ensure(g.tile_khi, nt * 8));
    RCCHK(ensure(g.tile_items, (nt + 1) * 8));
    RCCHK(ensure(g.counter, 64));
    RCCHK(ensure(g.pair_stats, 64));
    RCCHK(ensure(g.out_dev, nq * 8));

    hipStream_t s = g.stream;
    HIPCHK(hipMemcpyAsync(g.q_n.p, ns.data(), nq * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(g.q_L.p, Ls.data(), nq * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(g.q_g0.p, g0s.data(), nq * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(g.tile_q.p, t_q.data(), nt * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(g.tile_x0.p, t_x0.data(), nt * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(g.tile_nx.p, t_nx.data(), nt * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(g.tile_g0.p, t_g0.data(), nt * 8, hipMemcpyHostToDevice, s));

    QueryArgs q;
    q.nq = (uint32_t)nq;
    q.q_n = g.q_n.as<uint64_t>();
    q.q_L = g.q_L.as<uint64_t>();
    q.q_g0 = g.q_g0.as<uint64_t>();
    q.x_m = g.x_m.as<uint64_t>();
    q.x_Y = g.x_Y.as<uint64_t>();
    q.x_K = g.x_K.as<uint64_t>();
    q.x_k0 = g.x_k0.as<uint64_t>();
    q.S = g.S.as<uint64_t>();
    q.A = g.A.as<int64_t>();
    q.x_klo = g.x_klo.as<uint64_t>();
    q.x_khi = g.x_khi.as<uint64_t>();
    q.ntiles = (uint32_t)nt;
    q.tile_q = g.tile_q.as<uint32_t>();
    q.tile_x0 = g.tile_x0.as<uint32_t>();
    q.tile_nx = g.tile_nx.as<uint32_t>();
    q.tile_g0 = g.tile_g0.as<uint64_t>();
    q.tile_ymax = g.tile_ymax.as<uint64_t>();
    q.tile_klo = g.tile_klo.as<uint64_t>();
    q.tile_khi = g.tile_khi.as<uint64_t>();
    q.tile_mode = g.tile_mode.as<uint32_t>();
    q.tile_nmu = g.tile_nmu.as<uint32_t>();
    q.tile_items = g.tile_items.as<uint64_t>();
    q.counter = g.counter.as<uint32_t>();
    q.pair_stats = g.pair_stats.as<uint64_t>();
    q.beta = g.beta;
    q.ychunk = g.ychunk;
    q.kchunk = g.kchunk;
    q.klchunk = g.klchunk;

    const uint64_t nblocks = ymax / B + 1;
    size_t ev = 0;
    hipEvent_t e_start = event_at(ev++);
    if (!e_start) {
        set_error_text("hipEventCreate failed");
        return MERTENS_EIO;
    }
    HIPCHK(hipEventRecord(e_start, s));
    HIPCHK(launch_zero_u64(g.pair_stats.as<uint64_t>(), 4, s));
    HIPCHK(launch_zero_u64(reinterpret_cast<uint64_t *>(g.carry.p), 1, s));
    HIPCHK(launch_plan(q, s));
    const uint32_t grid = (uint32_t)std::max(1, g.ncu * (int)g.waves_per_cu / (UPD_THREADS / 64));
    std::vector<size_t> marks;
    marks.reserve(nblocks * 5);
    for (uint64_t bi = 0; bi < nblocks; ++bi) {
        const uint64_t y1 = bi * B;
        const uint64_t y2 = std::min(y1 + B - 1, ymax);
        const BlockArgs b = make_block(y1, y2);
        hipEvent_t e0 = event_at(ev), e1 = event_at(ev + 1), e2 = event_at(ev + 2),
                   e3 = event_at(ev + 3), e4 = event_at(ev + 4);
        if (!e0 || !e1 || !e2 || !e3 || !e4) {
            set_error_text("hipEventCreate failed");
            return MERTENS_EIO;
        }
        marks.push_back(ev);
        ev += 5;
        RCCHK(sieve_block(b, e0));
        HIPCHK(hipEventRecord(e1, s));
        RCCHK(scan_block(b));
        HIPCHK(hipEventRecord(e2, s));
        HIPCHK(launch_update_prep(q, b, s));
        HIPCHK(launch_scan_items(q, s));
        HIPCHK(hipEventRecord(e3, s));
        HIPCHK(launch_update(q, b, grid, s));
        HIPCHK(hipEventRecord(e4, s));
    }
    hipEvent_t ef0 = event_at(ev), ef1 = event_at(ev + 1);
    if (!ef0 || !ef1) {
        set_error_text("hipEventCreate failed");
        return MERTENS_EIO;
    }
    HIPCHK(hipEventRecord(ef0, s));
    HIPCHK(launch_finalize(q, s));
    HIPCHK(hipEventRecord(ef1, s));
    HIPCHK(launch_collect(q, g.out_dev.as<int64_t>(), s));
    res.resize(nq);
    uint64_t pst[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(res.data(), g.out_dev.p, nq * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(pst, g.pair_stats.p, 32, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));

    double t_sieve = 0, t_scan = 0, t_prep = 0, t_upd = 0;
    for (size_t m : marks) {
        t_sieve += elapsed(m, m + 1);
        t_scan += elapsed(m + 1, m + 2);
        t_prep += elapsed(m + 2, m + 3);
        t_upd += elapsed(m + 3, m + 4);
    }
    g.stats[0] = (double)(ymax + 1);
    g.stats[1] = (double)nblocks;
    g.stats[2] = (double)u;
    g.stats[3] = (double)X;
    g.stats[4] = (double)pst[0];
    g.stats[5] = (double)pst[1];
    g.stats[6] = t_sieve;
    g.stats[7] = t_scan;
    g.stats[8] = t_prep;
    g.stats[9] = t_upd;
    g.stats[10] = elapsed(ev, ev + 1);
    g.stats[11] = elapsed(0, ev + 1);
    g.stats[12] = (double)nblocks;
    g.stats[13] = (double)nblocks;
    g.stats[14] = (double)pst[2];
    g.stats[15] = (double)pst[3];
    return 0;
}

}  // namespace

// ======================================================================
// C ABI
// ======================================================================
extern "C" {

int mertens_init(uint64_t u, uint64_t block)
{
    if (block != 0 && (block < SEG || block % SEG != 0 || block > (1ull << 31))) {
        set_error_text("block must be 0 or a multiple of 131072 in [131072, 2^31]");
        return MERTENS_EINVAL;
    }
    if (g.ready)
        free_all();
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        set_error_text("no HIP device");
        return MERTENS_ENODEV;
    }
    HIPCHK(hipGetDevice(&g.device));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, g.device));
    g.ncu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    HIPCHK(hipStreamCreateWithFlags(&g.own_stream, hipStreamNonBlocking));
    g.stream = g.own_stream;
    g.u_req = u;
    g.block_req = block;
    int rc = upload_pattern();
    if (rc == 0)
        rc = ensure_primes(1024);
    if (rc != 0) {
        free_all();
        return rc;
    }
    g.ready = true;
    return 0;
}

int mertens_query(const uint64_t *n, size_t count, int64_t *out)
{
    if (count == 0)
        return 0;
    if (!n || !out) {
        set_error_text("null pointer with count > 0");
        return MERTENS_EINVAL;
    }
    if (!g.ready) {
        set_error_text("mertens_init has not been called");
        return MERTENS_ENODEV;
    }
    std::vector<uint64_t> ns;
    std::vector<size_t> where;
    for (size_t i = 0; i < count; ++i)
        if (n[i] != 0) {
            ns.push_back(n[i]);
            where.push_back(i);
        }
    std::vector<int64_t> res;
    std::vector<uint64_t> Ls, g0s;
    g.last_valid = false;
    if (!ns.empty()) {
        int rc = run_query(ns, res, Ls, g0s);
        if (rc != 0)
            return rc;
    }
    g.last_L.assign(count, 0);
    g.last_g0.assign(count, 0);
    for (size_t i = 0; i < count; ++i)
        out[i] = 0;
    for (size_t j = 0; j < where.size(); ++j) {
        out[where[j]] = res[j];
        g.last_L[where[j]] = Ls[j];
        g.last_g0[where[j]] = g0s[j];
    }
    g.last_valid = true;
    return 0;
}

int mertens_byproducts(size_t i, int64_t *buf, size_t cap, size_t *len)
{
    if (!g.ready)
        return MERTENS_ENODEV;
    if (!g.last_valid || i >= g.last_L.size())
        return MERTENS_ERANGE;
    if (cap > 0 && !buf)
        return MERTENS_EINVAL;
    const uint64_t L = g.last_L[i];
    if (len)
        *len = (size_t)L;
    const size_t k = (size_t)std::min<uint64_t>(L, cap);
    if (k > 0) {
        HIPCHK(hipMemcpyAsync(buf, g.A.as<int64_t>() + g.last_g0[i], k * 8, hipMemcpyDeviceToHost,
                              g.stream));
        HIPCHK(hipStreamSynchronize(g.stream));
    }
    return 0;
}

int mertens_set_stream(void *hip_stream)
{
    if (!g.ready)
        return MERTENS_ENODEV;
    g.stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : g.own_stream;
    return 0;
}

int mertens_set_param(const char *key, double value)
{
    if (!key)
        return MERTENS_EINVAL;
    if (!strcmp(key, "beta")) {
        if (!(value > 0.0 && value <= 1.0))
            return MERTENS_EINVAL;
        g.beta = value;
    } else if (!strcmp(key, "ychunk")) {
        if (!(value >= 64 && value <= (1 << 24)) || ((uint64_t)value) % 64 != 0)
            return MERTENS_EINVAL;
        g.ychunk = (uint32_t)value;
    } else if (!strcmp(key, "kchunk")) {
        if (!(value >= 64 && value <= (1 << 24)))
            return MERTENS_EINVAL;
        g.kchunk = (uint32_t)value;
    } else if (!strcmp(key, "klchunk")) {
        if (!(value >= 1 && value <= (1 << 24)))
            return MERTENS_EINVAL;
        g.klchunk = (uint32_t)value;
    } else if (!strcmp(key, "waves_per_cu")) {
        if (!(value >= 4 && value <= 64))
            return MERTENS_EINVAL;
        g.waves_per_cu = (uint32_t)value;
    } else {
        return MERTENS_EINVAL;
    }
    return 0;
}

int mertens_stats(double *vals, int cap)
{
    if (!vals || cap <= 0)
        return 0;
    const int k = std::min(cap, 16);
    for (int i = 0; i < k; ++i)
        vals[i] = g.stats[i];
    return k;
}

void mertens_shutdown(void)
{
    if (g.ready)
        (void)hipStreamSynchronize(g.stream);
    free_all();
}

const char *mertens_strerror(int code)
{
    switch (code) {
    case 0: return "success";
    case MERTENS_EINVAL: return "invalid argument";
    case MERTENS_ENOMEM: return "out of memory";
    case MERTENS_ENODEV: return "no device or not initialised";
    case MERTENS_ERANGE: return "index out of range";
    case MERTENS_EIO: return "HIP runtime error";
    case MERTENS_EAGAIN: return "no free slot";
    case MERTENS_EINPROGRESS: return "in progress";
    default: return "unknown error";
    }
}

const char *mertens_last_error(void) { return g_last_error.c_str(); }

int mertens_debug_div(const uint64_t *n, const uint64_t *d, size_t count, uint64_t *q,
                      int on_device)
{
    if (count == 0)
        return 0;
    if (!n || !d || !q)
        return MERTENS_EINVAL;
    for (size_t i = 0; i < count; ++i)
        if (d[i] == 0 || d[i] >= (1ull << 32))
            return MERTENS_EINVAL;
    if (!on_device) {
        for (size_t i = 0; i < count; ++i) {
            uint64_t mul;
            uint32_t s1, s2;
            host_magic((uint32_t)d[i], &mul, &s1, &s2);
            q[i] = host_div(n[i], mul, s1, s2);
        }
        return 0;
    }
    if (!g.ready)
        return MERTENS_ENODEV;
    DevBuf dn, dd, dq;
    int rc = ensure(dn, count * 8);
    if (!rc)
        rc = ensure(dd, count * 8);
    if (!rc)
        rc = ensure(dq, count * 8);
    if (!rc) {
        hipError_t e = hipMemcpy(dn.p, n, count * 8, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(dd.p, d, count * 8, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_debug_div(dn.as<uint64_t>(), dd.as<uint64_t>(), dq.as<uint64_t>(), count,
                                 g.stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(g.stream);
        if (e == hipSuccess)
            e = hipMemcpy(q, dq.p, count * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            set_error("debug_div", e, __FILE__, __LINE__);
            rc = MERTENS_EIO;
        }
    }
    dn.release();
    dd.release();
    dq.release();
    return rc;
}

int mertens_debug_mu(uint64_t y1, size_t count, int8_t *mu, int64_t *mert)
{
    if (count == 0)
        return 0;
    if (!mu || count > (1ull << 31) || y1 > (1ull << 63) - count)
        return MERTENS_EINVAL;
    if (!g.ready)
        return MERTENS_ENODEV;
    const uint64_t yend = y1 + count - 1;
    const uint64_t start = y1 - y1 % SEG;
    RCCHK(ensure_primes(std::max<uint64_t>(ceil_sqrt_host(yend), 1024)));
    const uint64_t B = 1ull << 30;
    RCCHK(ensure_block_buffers(B));
    DevBuf dmu, dm;
    int rc = ensure(dmu, count);
    if (!rc)
        rc = ensure(dm, count * 8);
    if (rc) {
        dmu.release();
        dm.release();
        return rc;
    }
    hipError_t e = launch_zero_u64(reinterpret_cast<uint64_t *>(g.carry.p), 1, g.stream);
    for (uint64_t y = start; e == hipSuccess && y <= yend; y += B) {
        const uint64_t y2 = std::min(y + B - 1, yend);
        const BlockArgs b = make_block(y, y2);
        if (sieve_block(b) != 0 || scan_block(b) != 0) {
            e = hipErrorUnknown;
            break;
        }
        const uint64_t lo = std::max(y, y1);
        e = launch_debug_mu(b, lo, (uint32_t)(y2 - lo + 1), dmu.as<int8_t>() + (lo - y1),
                            dm.as<int64_t>() + (lo - y1), g.stream);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(g.stream);
    std::vector<int64_t> hm;
    if (e == hipSuccess)
        e = hipMemcpy(mu, dmu.p, count, hipMemcpyDeviceToHost);
    if (e == hipSuccess && mert) {
        hm.resize(count);
        e = hipMemcpy(hm.data(), dm.p, count * 8, hipMemcpyDeviceToHost);
    }
    dmu.release();
    dm.release();
    if (e != hipSuccess) {
        set_error("debug_mu", e, __FILE__, __LINE__);
        return MERTENS_EIO;
    }
    if (mert) {
        // device values are sums from `start`; the window sums start at y1
        const int64_t before = hm[0] - (int64_t)mu[0];
        for (size_t i = 0; i < count; ++i)
            mert[i] = hm[i] - before;
    }
    return 0;
}

}  // extern "C"
