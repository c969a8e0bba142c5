// Host runtime and C ABI of the gfx950 Mertens library (see include/mertens.h).
//
// Two engines share the same building blocks:
//   * the synchronous path (mertens_query): one Batch of queries, one sweep
//     over y-blocks 0, 1, ... in order, then finalize;
//   * the serving path (mertens_submit / mertens_poll): a worker thread runs
//     a cyclic sweep; requests join at the next block boundary as a new
//     Batch, each query completes once every block it needs has been
//     visited once since it joined (contributions commute, so the order of
//     blocks does not matter; within a pass the sieve carry runs in
//     ascending y), and is finalized and returned on its own.
// Per block the kernel sequence is (Section 3):
//   residues -> sieve with fused M(y) prefix -> update prep -> item prefix
//   -> persistent update
// with no host synchronisation inside a sweep.
#include "mertens.h"
#include "mertens_internal.h"

#include <dlfcn.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

using namespace mrt;

namespace {

std::mutex g_err_mu;
std::string g_last_error = "no error";

void set_error(const char *what, hipError_t e, const char *file, int line)
{
    char buf[512];
    snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    std::lock_guard<std::mutex> lk(g_err_mu);
    g_last_error = buf;
}

void set_error_text(const char *text)
{
    std::lock_guard<std::mutex> lk(g_err_mu);
    g_last_error = text;
}

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

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool owned = true;  // false: a piece of the no-alloc scratch (never freed)
    template <class T>
    T *as() const { return static_cast<T *>(p); }
    void release()
    {
        if (p && owned)
            (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        owned = true;
    }
};

// While `on`, every buffer is carved from the no-alloc scratch (the device
// address of the `scratch` array, 256-byte pieces) instead of hipMalloc.
struct Arena {
    uint8_t *base = nullptr;
    size_t cap = 0, used = 0;
    bool on = false;
};
Arena g_arena;

int ensure(DevBuf &b, size_t bytes)
{
    if (bytes < 64)
        bytes = 64;
    if (g_arena.on) {
        if (b.bytes >= bytes && !b.owned)
            return 0;
        const size_t at = (g_arena.used + 255) & ~(size_t)255;
        if (b.owned && b.p) {
            set_error_text("no-alloc call would have to free a device buffer");
            return MERTENS_EINVAL;
        }
        if (at > g_arena.cap || bytes > g_arena.cap - at) {
            set_error_text("the request needs more device memory than the no-alloc scratch holds");
            return MERTENS_ENOMEM;
        }
        b.p = g_arena.base + at;
        b.bytes = bytes;
        b.owned = false;
        g_arena.used = at + bytes;
        return 0;
    }
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

// scale * N^(2/3): with a sieve cost proportional to u and an update cost
// proportional to (sum of n)/sqrt(u), the total is smallest at u ~ (sum n)^(2/3)
// (Section 2, and its remark on several close values of n); the scale is
// the tuned ratio of the two costs.
// Sum of n over clusters of nearly equal n (consecutive sorted values within
// a relative 2^-20 of the cluster's first): such queries share L and one
// keyed set of entries, so their update costs about one query's.
long double effective_total_n(std::vector<uint64_t> v)
{
    std::sort(v.begin(), v.end());
    long double sum = 0;
    size_t i = 0;
    while (i < v.size()) {
        const uint64_t start = v[i];
        size_t j = i + 1;
        while (j < v.size() && v[j] - start <= (start >> 20))
            ++j;
        sum += (long double)v[j - 1];
        i = j;
    }
    return sum;
}

uint64_t auto_u(long double total_n, double scale)
{
    const double v = scale * std::pow((double)total_n, 2.0 / 3.0);
    uint64_t u = (uint64_t)std::ceil(v > 1.8e19 ? 1.8e19 : v);
    return u < 2 ? 2 : u;
}

struct Tuning {
    double u_scale = 0.5;  // automatic u = u_scale * (clustered sum of the batch's n)^(2/3)
    double beta = 0.25;
    uint32_t ychunk = 16384, kchunk = 1024, waves_per_cu = 12;  // 3 update workgroups per CU
    uint32_t kbal = 0;  // 0: every tile takes the 8 x 8 walk (measured best at 1e16)
    uint32_t sieve_ahead = 4;  // most record slots (blocks sieved ahead of the update)
    // blocks starting below window_ymax are updated in windows of
    // 2^update_window y, so the records that the explicit-k gathers of one
    // window touch stay cache-resident (0: whole blocks)
    uint32_t update_window = 0;
    uint64_t window_ymax = 1ull << 30;
    uint32_t rl_fast = 1;
    // explicit-k pairs with quotients in [2^band_lo, 2^band_hi) are summed
    // y-major from LDS windows of the records (k_ek_window), the rest by the
    // persistent update (band_lo = 0: none)
    uint32_t band_lo = 20, band_hi = 28;
    // x with floor(n/x) >= 2^wide_bits go through the 128-bit wide entries
    // (64: exactly those that need more than 64 bits)
    uint32_t wide_bits = 64;
    // > 0: wait for every progress-th block of a query and report it on
    // stderr (for sweeps that run many minutes)
    uint64_t progress = 0;
    bool graph = false;  // replay one captured hipGraph per block
    uint64_t block_auto = 1ull << 30;  // block length when mertens_init gets block = 0
};

// The band of explicit-k quotients that block [y1, y2] sums y-major, as
// the window range [ys, ye): none when the band is off or misses the block,
// or when its windows would not start at a multiple of their length.
bool band_of(const Tuning &t, uint64_t y1, uint64_t y2, uint64_t &ys, uint64_t &ye)
{
    if (t.band_lo < EKW_SHIFT || t.band_hi <= t.band_lo || t.band_hi > 31)
        return false;
    ys = std::max<uint64_t>(1ull << t.band_lo, y1);
    ye = std::min<uint64_t>(1ull << t.band_hi, y2 + 1);
    return ys < ye && ys % (1ull << EKW_SHIFT) == 0;
}

#ifndef MERTENS_KERNEL_SHA256
#define MERTENS_KERNEL_SHA256 ""
#endif
#ifndef MERTENS_ARCH_NAME
#define MERTENS_ARCH_NAME "gfx950"
#endif

// Primes p in [5, limit] (limit <= 2^32) into pr, ascending: segmented
// Eratosthenes over odd numbers, 2^19 of them per segment, crossed off by the
// base primes up to sqrt(limit).  Large limits split the segments over up to
// 16 host threads (contiguous runs, joined in order).
void host_primes(uint64_t limit, std::vector<uint32_t> &pr)
{
    pr.clear();
    const uint64_t root = isqrt_host(limit);
    std::vector<uint8_t> bc(root / 2 + 1, 0);  // bc[i] <=> 2i+1 composite, 2i+1 <= root
    std::vector<uint32_t> base;
    for (uint64_t i = 3; i <= root; i += 2)
        if (!bc[i / 2]) {
            base.push_back((uint32_t)i);
            for (uint64_t j = i * i; j <= root; j += 2 * i)
                bc[j / 2] = 1;
        }
    constexpr uint64_t SPAN = 1ull << 19;  // odd numbers per segment
    const uint64_t nseg = limit / (2 * SPAN) + 1;
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const uint64_t nthr = limit < (1ull << 26) ? 1 : std::min<uint64_t>(hw, nseg);
    std::vector<std::vector<uint32_t>> part(nthr);
    auto work = [&](uint64_t t) {
        std::vector<uint8_t> comp(SPAN);
        std::vector<uint32_t> &out = part[t];
        const uint64_t s0 = nseg * t / nthr, s1 = nseg * (t + 1) / nthr;
        for (uint64_t sg = s0; sg < s1; ++sg) {
            const uint64_t lo = 1 + sg * 2 * SPAN;  // odd v in [lo, lo + 2 SPAN)
            if (lo > limit)
                break;
            std::fill(comp.begin(), comp.end(), 0);
            const uint64_t hi = std::min(lo + 2 * SPAN - 1, limit);
            for (uint32_t q : base) {
                const uint64_t qq = (uint64_t)q * q;
                if (qq > hi)
                    break;
                uint64_t f = std::max(qq, (lo + q - 1) / q * q);
                if (f % 2 == 0)
                    f += q;
                for (uint64_t v = f; v <= hi; v += 2 * q)
                    comp[(v - lo) / 2] = 1;
            }
            for (uint64_t v = std::max<uint64_t>(lo, 5); v <= hi; v += 2)
                if (!comp[(v - lo) / 2])
                    out.push_back((uint32_t)v);
        }
    };
    if (nthr == 1) {
        work(0);
    } else {
        std::vector<std::thread> th;
        for (uint64_t t = 0; t < nthr; ++t)
            th.emplace_back(work, t);
        for (std::thread &x : th)
            x.join();
    }
    size_t total = 0;
    for (const auto &v : part)
        total += v.size();
    pr.reserve(total);
    for (const auto &v : part)
        pr.insert(pr.end(), v.begin(), v.end());
}

// ---------------------------------------------------------------------------
// Device tables and block buffers of one sweep engine.
// ---------------------------------------------------------------------------
struct SieveState {
    uint64_t psieve = 0;
    std::vector<uint32_t> h_primes;  // primes >= 5 up to psieve
    DevBuf pres, res2, pattern, words, seg_state, sq_cnt, sq_buf, bk_cnt, bk_start, bk_buf,
        bk_stage, carry, bp_cur, bp_table, bp_index;
    uint32_t bucket_min = 1u << 20;  // bucket the primes above SEG when a block has this many
    long double bk_cap = 0;           // bucket entries a block of bk_cap_B can need
    uint64_t bk_cap_B = 0, bk_cap_np = 0;
    bool have_pattern = false;

    void release()
    {
        DevBuf *bufs[] = {&pres, &res2, &pattern, &words, &seg_state, &sq_cnt, &sq_buf,
                          &bk_cnt, &bk_start, &bk_buf, &bk_stage, &carry, &bp_cur, &bp_table,
                          &bp_index};
        for (DevBuf *b : bufs)
            b->release();
        h_primes.clear();
        psieve = 0;
        have_pattern = false;
    }

    // Sieving primes p in [5, limit] (host_primes) and their device copy as
    // {p, residue} pairs.  Grows only, by at least a quarter at a time.
    int ensure_primes(uint64_t limit)
    {
        if (limit <= psieve)
            return 0;
        if (psieve)  // grow by at least a quarter, so rising limits re-sieve rarely
            limit = std::max(limit, std::min<uint64_t>(psieve + psieve / 4, 1ull << 32));
        std::vector<uint32_t> pr;
        host_primes(limit, pr);
        const size_t np = pr.size();
        std::vector<uint32_t> pairs(2 * np, 0u);
        for (size_t i = 0; i < np; ++i)
            pairs[2 * i] = pr[i];
        RCCHK(ensure(pres, np * 8));
        RCCHK(ensure(res2, np * 8));
        HIPCHK(hipMemcpy(pres.p, pairs.data(), np * 8, hipMemcpyHostToDevice));
        h_primes.swap(pr);
        psieve = limit;
        return 0;
    }

    // Pattern of the modified sieve for the primes 2, 3, 5, 7, 11, 13 and the
    // squares 4, 9 (period 180180), extended by one segment so a segment's
    // initial state is one straight copy, in the sieve's LDS layout (y
    // offset q of a copy at byte (q & ~31) | (q & 7) << 2 | (q >> 3) & 3),
    // in eight copies, copy c starting at pattern byte 4c.
    int ensure_pattern()
    {
        if (have_pattern)
            return 0;
        const uint32_t small[6] = {2, 3, 5, 7, 11, 13};
        const size_t copy_bytes = (size_t)PAT_WORDS * 4;
        std::vector<uint8_t> pat(copy_bytes * PAT_COPIES, 0);
        for (size_t c = 0; c < PAT_COPIES; ++c) {
            for (size_t q = 0; q < copy_bytes; ++q) {
                const uint32_t r = (uint32_t)((4 * c + q) % PAT);
                uint32_t a = 0;
                for (uint32_t p : small)
                    if (r % p == 0)
                        a += log_prime_host(p);
                if (r % 4 == 0 || r % 9 == 0)
                    a |= 0x80u;
                const size_t at = (q & ~(size_t)31) | ((q & 7) << 2) | ((q >> 3) & 3);
                pat[c * copy_bytes + at] = (uint8_t)a;
            }
        }
        RCCHK(ensure(pattern, pat.size()));
        HIPCHK(hipMemcpy(pattern.p, pat.data(), pat.size(), hipMemcpyHostToDevice));
        have_pattern = true;
        return 0;
    }

    // The pattern of another state (already on the device), copied on the
    // device (the no-alloc path takes its copy into the scratch this way).
    int copy_pattern(const DevBuf &src, hipStream_t s)
    {
        RCCHK(ensure(pattern, src.bytes));
        HIPCHK(hipMemcpyAsync(pattern.p, src.p, src.bytes, hipMemcpyDeviceToDevice, s));
        have_pattern = true;
        return 0;
    }

    // record buffers for `slots` blocks of length B (a ring: block b uses
    // slot b mod slots) and their per-slot device parameters, followed by
    // the parameters of up to MAX_WINDOWS update windows
    static constexpr uint32_t MAX_WINDOWS = 1024;
    uint32_t slots = 1;
    uint64_t slot_words = 0;  // uint64 per slot

    int ensure_blocks(uint64_t B, uint32_t nslots = 1)
    {
        RCCHK(ensure(words, (size_t)nslots * (B / 64 * 32)));
        slots = nslots;
        slot_words = B / 64 * 4;
        RCCHK(ensure(seg_state, B / SEG * 8));
        RCCHK(ensure(sq_cnt, B / SEG * 4));
        RCCHK(ensure(sq_buf, B / SEG * SQ_BUCKET * 4));
        // bucketed primes: counts, starts, and every multiple in a block of
        // any prime above SEG (at most B / p + 1 each)
        const uint32_t n_mid = count_primes_upto(SEG);
        if (bucketed(h_primes.size(), psieve)) {
            if (bk_cap_B != B || bk_cap_np != h_primes.size()) {
                long double c = 0;
                for (size_t i = n_mid; i < h_primes.size(); ++i)
                    c += (long double)B / h_primes[i] + 1;
                bk_cap = c;
                bk_cap_B = B;
                bk_cap_np = h_primes.size();
            }
            const long double cap = bk_cap;
            if (cap >= 4.0e9L) {
                set_error_text("too many bucketed multiples per block; use a smaller block");
                return MERTENS_EINVAL;
            }
            RCCHK(ensure(bk_cnt, (size_t)BK_WGS * (B / SEG) * 4));
            RCCHK(ensure(bk_start, (B / SEG + 1) * 4));
            RCCHK(ensure(bk_buf, (size_t)cap * 4 + 64));
            RCCHK(ensure(bk_stage, (size_t)cap * 4 + 64));
        }
        // M(y1 - 1) at byte 0, segment ticket at byte 8, bucket entry count at 16
        RCCHK(ensure(carry, 64));
        RCCHK(ensure(bp_cur, ((size_t)nslots + MAX_WINDOWS) * sizeof(BlockParams)));
        RCCHK(ensure(bp_index, 64));
        return 0;
    }

    // Whether a block whose n_sieve sieving primes reach pmax lists the
    // multiples of its primes above SEG in buckets: when there are
    // bucket_min of them, or when they outnumber the multiples they leave in
    // a segment (SEG times the sum of 1/p over (SEG, pmax], by Mertens'
    // second theorem about SEG ln(ln pmax / ln SEG)) BK_RATIO times or more:
    // without buckets each such prime costs a residue in every segment,
    // with them each multiple costs a listed entry.
    static constexpr double BK_RATIO = 8.0;
    bool bucketed(uint64_t n_sieve, uint64_t pmax) const
    {
        const uint64_t n_mid = count_primes_upto(SEG);
        if (n_sieve <= n_mid)
            return false;
        const uint64_t n_above = n_sieve - n_mid;
        if (n_above >= bucket_min)
            return true;
        const double hits = (double)SEG * std::log(std::log((double)pmax) / std::log((double)SEG));
        return (double)n_above >= BK_RATIO * hits;
    }

    uint32_t count_primes_upto(uint64_t v) const  // # table primes p <= v
    {
        return (uint32_t)(std::upper_bound(h_primes.begin(), h_primes.end(), v,
                                           [](uint64_t a, uint32_t b) { return a < b; }) -
                          h_primes.begin());
    }

    BlockArgs make_block(uint64_t y1, uint64_t y2, uint32_t slot = 0) const
    {
        BlockArgs b;
        b.bp = bp_cur.as<BlockParams>() + slot;
        b.y1 = y1;
        b.y2 = y2;
        b.nseg = (uint32_t)((y2 - y1) / SEG + 1);
        b.n_small = count_primes_upto(SMALL_P - 1);
        // primes up to sqrt(y2) decide mu on the block (and every p < SMALL_P)
        b.n_sieve = count_primes_upto(std::max<uint64_t>(ceil_sqrt_host(y2), SMALL_P));
        const uint32_t n_mid = count_primes_upto(SEG);
        b.n_bucket = bucketed(b.n_sieve, std::max<uint64_t>(ceil_sqrt_host(y2), SMALL_P)) ? n_mid
                                                                                        : b.n_sieve;
        b.n_lane = std::max(b.n_bucket, count_primes_upto((uint64_t)b.nseg * SEG / 64));
        b.n_lane = std::min(b.n_lane, b.n_sieve);
        b.bk_cnt = bk_cnt.as<uint32_t>();
        b.bk_start = bk_start.as<uint32_t>();
        b.bk_buf = bk_buf.as<uint32_t>();
        b.bk_stage = bk_stage.as<uint32_t>();
        b.n_sq = count_primes_upto(isqrt_host(y2));
        b.n_sq_lds = std::min(count_primes_upto(SQ_LDS_P), b.n_sq);
        b.n_sq_lane = std::min(std::max(count_primes_upto(isqrt_host((uint64_t)b.nseg * SEG / 64)),
                                        b.n_sq_lds),
                               b.n_sq);
        b.pat_off = (uint32_t)(y1 % PAT);
        b.pres = pres.as<uint2>();
        b.res2 = res2.as<uint64_t>();
        b.pat32 = pattern.as<uint32_t>();
        b.words = words.as<uint64_t>() + (size_t)slot * slot_words;
        b.seg_state = seg_state.as<uint64_t>();
        b.sq_cnt = sq_cnt.as<uint32_t>();
        b.sq_buf = sq_buf.as<uint32_t>();
        b.seg_ticket = reinterpret_cast<uint32_t *>(carry.as<uint8_t>() + 8);
        b.bk_total = reinterpret_cast<uint64_t *>(carry.as<uint8_t>() + 16);
        b.carry = carry.as<int64_t>();
        return b;
    }

    // Update window [ua, ub] (ua a multiple of 64) of block b: the same
    // records, addressed from ua, with its own device parameters.
    BlockArgs window_of(const BlockArgs &b, uint64_t ua, uint64_t ub, uint32_t w) const
    {
        BlockArgs v = b;
        v.words = b.words + (ua - b.y1) / 64 * 4;
        v.y1 = ua;
        v.y2 = ub;
        v.bp = bp_cur.as<BlockParams>() + slots + w;
        return v;
    }

    static BlockParams params_of(const BlockArgs &b)
    {
        BlockParams p;
        p.y1 = b.y1;
        p.y2 = b.y2;
        p.nseg = b.nseg;
        p.n_sq = b.n_sq;
        p.n_sq_lds = b.n_sq_lds;
        p.n_sq_lane = b.n_sq_lane;
        p.pat_off = b.pat_off;
        p.n_sieve = b.n_sieve;
        p.n_bucket = b.n_bucket;
        p.n_lane = b.n_lane;
        return p;
    }

    // Grid sizes that cover any block of length B (for the captured graph;
    // the kernels take the true values from the device parameters).
    BlockArgs max_block(uint64_t B) const
    {
        BlockArgs b = make_block(0, B - 1);
        b.nseg = (uint32_t)(B / SEG);
        b.n_sq_lds = 0;
        // grid sizes only: the wave kernel covers every n_sq_lane a block of
        // length <= B can have, the lane kernel every prime of the table
        b.n_sq_lane = count_primes_upto(isqrt_host(B / 64));
        b.n_sq = (uint32_t)h_primes.size() + b.n_sq_lane;
        b.n_sieve = (uint32_t)h_primes.size();
        // capture the bucket kernels whenever some block may use them
        const uint32_t n_mid = count_primes_upto(SEG);
        b.n_bucket = bucketed(b.n_sieve, psieve) ? n_mid : b.n_sieve;
        b.n_lane = std::min(std::max(b.n_bucket, count_primes_upto(B / 64)), b.n_sieve);
        return b;
    }

    // block parameters, residues and cleared scan state, then the sieve with
    // its fused M(y) prefix (an event may be recorded before it so the sieve
    // is timed alone).  set_params = false when a graph node loads the
    // parameters.
    int sieve(const BlockArgs &b, hipStream_t s, hipEvent_t between, bool set_params = true,
              hipEvent_t fill0 = nullptr, hipEvent_t fill1 = nullptr,
              hipEvent_t fill2 = nullptr) const
    {
        if (set_params)
            HIPCHK(launch_block_set(params_of(b), const_cast<BlockParams *>(b.bp), s));
        HIPCHK(launch_block_setup(b, s));
        HIPCHK(launch_square_buckets(b, s));
        HIPCHK(launch_prime_buckets(b, s, fill0, fill1, fill2));
        if (between)
            HIPCHK(hipEventRecord(between, s));
        HIPCHK(launch_sieve(b, s));
        return 0;
    }

    int reset_carry(hipStream_t s) const
    {
        HIPCHK(launch_zero_u64(reinterpret_cast<uint64_t *>(carry.p), 1, s));
        return 0;
    }
};

// ---------------------------------------------------------------------------
// One set of queries sharing a sweep: per-query plan and device state.
// ---------------------------------------------------------------------------
struct Batch {
    std::vector<uint64_t> n, nhi, xb, L, g0, ymax, koff;
    uint32_t nwide = 0;
    std::vector<uint32_t> fin_list;  // plain queries and one member per keyed group
    std::vector<uint32_t> key_off_h;  // host copy of key_off (keyed groups' levels)
    uint64_t X = 0, ymax_all = 0, keyed_entries = 0;
    uint32_t ntiles = 0;
    DevBuf q_n, q_L, q_g0, q_koff, x_m, x_Y, x_K, x_k0, S, A, x_klo, x_khi, key_x, key_off;
    DevBuf tile_q, tile_x0, tile_nx, tile_g0, tile_ymax, tile_klo, tile_khi, tile_mode, tile_nmu,
        tile_items, counter, pair_stats, out_dev, qlist, byp;
    DevBuf q_nhi, q_xb, w_g, w_x, w_q, w_mlo, w_mhi, w_K, w_Y, w_k0, w_klo, w_khi;
    QueryArgs args{};

    void release()
    {
        DevBuf *bufs[] = {&q_n, &q_L, &q_g0, &q_koff, &x_m, &x_Y, &x_K, &x_k0, &S, &A, &x_klo,
                          &x_khi, &key_x, &key_off, &tile_q, &tile_x0, &tile_nx, &tile_g0,
                          &tile_ymax, &tile_klo, &tile_khi, &tile_mode, &tile_nmu, &tile_items,
                          &counter, &pair_stats, &out_dev, &qlist, &byp, &q_nhi, &q_xb,
                          &w_g, &w_x, &w_q, &w_mlo, &w_mhi, &w_K, &w_Y, &w_k0, &w_klo, &w_khi};
        for (DevBuf *b : bufs)
            b->release();
    }

    // The distinct pairs (x, floor(v/x)) over the ascending values v[] for
    // x = 1..Lg, sorted by x then m, with the first entry of each x in off[]
    // (off[Lg] = number of entries).  Per x, the next value with a larger
    // quotient is found by binary search: work ~ entries * log(#values).
    static int make_keys(const std::vector<uint64_t> &v, uint64_t Lg, std::vector<uint32_t> &kx,
                         std::vector<uint64_t> &km, std::vector<uint32_t> &off)
    {
        kx.clear();
        km.clear();
        off.assign(Lg + 1, 0);
        for (uint64_t x = 1; x <= Lg; ++x) {
            if (km.size() >= 0xFFFFFFFFull) {
                set_error_text("too many distinct (x, n/x) entries in one group");
                return MERTENS_EINVAL;
            }
            off[x - 1] = (uint32_t)km.size();
            size_t i = 0;
            while (i < v.size()) {
                const uint64_t m = v[i] / x;
                kx.push_back((uint32_t)x);
                km.push_back(m);
                if (m + 1 > UINT64_MAX / x)
                    break;  // no value reaches (m+1) x
                const uint64_t next = (m + 1) * x;
                i = (size_t)(std::lower_bound(v.begin() + (ptrdiff_t)i + 1, v.end(), next) -
                             v.begin());
            }
        }
        off[Lg] = (uint32_t)km.size();
        return 0;
    }

    // Plan the queries ns[i] with split us[i] (Section 2: L = max(1, n/u)
    // array entries; the sieve covers [1, n/(L+1)]).  With `group`, queries
    // of equal L share one keyed set of entries (their contributions depend
    // on x and floor(n/x) only), so a dense window of n costs its distinct
    // quotients rather than one array per n.
    int plan(const std::vector<uint64_t> &ns, const std::vector<uint64_t> &us, const Tuning &t,
             hipStream_t s, bool group = true, const std::vector<uint64_t> *ns_hi = nullptr)
    {
        const size_t nq = ns.size();
        n = ns;
        nhi.assign(nq, 0);
        if (ns_hi)
            nhi = *ns_hi;
        xb.assign(nq, 0);
        bool wide = t.wide_bits < 64;
        for (uint64_t h : nhi)
            wide = wide || h != 0;
        group = group && !wide;  // keyed groups take 64-bit arguments only
        L.assign(nq, 0);
        g0.assign(nq, 0);
        ymax.assign(nq, 0);
        koff.assign(nq, ~0ull);
        fin_list.clear();
        X = 0;
        ymax_all = 0;
        keyed_entries = 0;
        for (size_t i = 0; i < nq; ++i) {
            const unsigned __int128 N = ((unsigned __int128)nhi[i] << 64) | ns[i];
            const unsigned __int128 Lw = N / us[i];
            if (Lw >= (1ull << 31)) {
                set_error_text("u too small: some n would need an array of 2^31 or more entries");
                return MERTENS_EINVAL;
            }
            const uint64_t Li = Lw < 1 ? 1 : (uint64_t)Lw;
            L[i] = Li;
            const unsigned __int128 ym = N / (Li + 1);
            if (ym >> 62) {
                set_error_text("u too large: the sieve bound n/(L+1) must stay below 2^62");
                return MERTENS_EINVAL;
            }
            ymax[i] = (uint64_t)ym;
            ymax_all = std::max(ymax_all, ymax[i]);
            const unsigned __int128 nb = N >> t.wide_bits;  // x <= nb have m >= 2^wide_bits
            xb[i] = nb < Li ? (uint64_t)nb : Li;
        }
        // groups of equal L (ascending n inside a group)
        std::vector<size_t> order(nq);
        for (size_t i = 0; i < nq; ++i)
            order[i] = i;
        if (group)
            std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
                return L[a] != L[b] ? L[a] < L[b] : ns[a] < ns[b];
            });
        std::vector<uint32_t> t_q, t_x0, t_nx;
        std::vector<uint64_t> t_g0;
        struct KeyedGroup {
            uint64_t g0;
            std::vector<uint32_t> kx;
            std::vector<uint64_t> km;
        };
        std::vector<KeyedGroup> kgroups;
        std::vector<uint32_t> h_key_off;
        for (size_t a = 0; a < nq;) {
            size_t b = a + 1;
            while (group && b < nq && L[order[b]] == L[order[a]])
                ++b;
            const uint64_t Lg = L[order[a]];
            if (b - a == 1) {
                const size_t i = order[a];
                g0[i] = X;
                fin_list.push_back((uint32_t)i);
                for (uint64_t x0 = 1; x0 <= Lg; x0 += TILE) {
                    t_q.push_back((uint32_t)i);
                    t_x0.push_back((uint32_t)x0);
                    t_nx.push_back((uint32_t)std::min<uint64_t>(TILE, Lg - x0 + 1));
                    t_g0.push_back(X + x0 - 1);
                }
                X += Lg;
            } else {
                std::vector<uint64_t> v;
                for (size_t j = a; j < b; ++j)
                    v.push_back(ns[order[j]]);
                KeyedGroup kg;
                kg.g0 = X;
                std::vector<uint32_t> off;
                RCCHK(make_keys(v, Lg, kg.kx, kg.km, off));
                const uint64_t base = h_key_off.size();
                h_key_off.insert(h_key_off.end(), off.begin(), off.end());
                for (size_t j = a; j < b; ++j) {
                    g0[order[j]] = X;
                    koff[order[j]] = base;
                }
                fin_list.push_back((uint32_t)order[a]);
                const uint64_t E = kg.km.size();
                for (uint64_t e = 0; e < E; e += TILE) {
                    t_q.push_back((uint32_t)order[a]);
                    t_x0.push_back(0u);
                    t_nx.push_back((uint32_t)std::min<uint64_t>(TILE, E - e));
                    t_g0.push_back(X + e);
                }
                X += E;
                keyed_entries += E;
                kgroups.push_back(std::move(kg));
            }
            a = b;
        }
        // wide entries: x = 1..xb of every query
        std::vector<uint64_t> h_wg;
        std::vector<uint32_t> h_wx, h_wq;
        for (size_t i = 0; i < nq; ++i)
            for (uint64_t x = 1; x <= xb[i]; ++x) {
                if (h_wg.size() >= (1u << 24)) {
                    set_error_text("too many wide entries (x with floor(n/x) >= 2^wide_bits)");
                    return MERTENS_EINVAL;
                }
                h_wg.push_back(g0[i] + x - 1);
                h_wx.push_back((uint32_t)x);
                h_wq.push_back((uint32_t)i);
            }
        nwide = (uint32_t)h_wg.size();
        if (nwide && ymax_all >= (1ull << 50)) {
            set_error_text("wide arguments need a sieve bound n/(L+1) below 2^50");
            return MERTENS_EINVAL;
        }
        const size_t nt = t_q.size();
        if (nt >= (1ull << 31)) {
            set_error_text("too many tiles");
            return MERTENS_EINVAL;
        }
        ntiles = (uint32_t)nt;
        RCCHK(ensure(q_n, nq * 8));
        RCCHK(ensure(q_L, nq * 8));
        RCCHK(ensure(q_g0, nq * 8));
        RCCHK(ensure(q_koff, nq * 8));
        DevBuf *xbufs[] = {&x_m, &x_Y, &x_K, &x_k0, &S, &A, &x_klo, &x_khi};
        for (DevBuf *b : xbufs)
            RCCHK(ensure(*b, X * 8));
        RCCHK(ensure(key_x, std::max<uint64_t>(X, 1) * 4));
        RCCHK(ensure(key_off, std::max<size_t>(h_key_off.size(), 1) * 4));
        RCCHK(ensure(tile_q, nt * 4));
        RCCHK(ensure(tile_x0, nt * 4));
        RCCHK(ensure(tile_nx, nt * 4));
        RCCHK(ensure(tile_mode, nt * 4));
        RCCHK(ensure(tile_nmu, nt * 4));
        RCCHK(ensure(tile_g0, nt * 8));
        RCCHK(ensure(tile_ymax, nt * 8));
        RCCHK(ensure(tile_klo, nt * 8));
        RCCHK(ensure(tile_khi, nt * 8));
        RCCHK(ensure(tile_items, (nt + 1) * 8));
        RCCHK(ensure(counter, 64));
        RCCHK(ensure(pair_stats, 64));
        RCCHK(ensure(out_dev, nq * 8));
        RCCHK(ensure(qlist, nq * 4));
        RCCHK(ensure(q_nhi, nq * 8));
        RCCHK(ensure(q_xb, nq * 8));
        const size_t nw1 = std::max<size_t>(nwide, 1);
        DevBuf *wb[] = {&w_g, &w_mlo, &w_mhi, &w_K, &w_Y, &w_k0, &w_klo, &w_khi};
        for (DevBuf *b : wb)
            RCCHK(ensure(*b, nw1 * 8));
        RCCHK(ensure(w_x, nw1 * 4));
        RCCHK(ensure(w_q, nw1 * 4));
        HIPCHK(hipMemcpyAsync(q_nhi.p, nhi.data(), nq * 8, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(q_xb.p, xb.data(), nq * 8, hipMemcpyHostToDevice, s));
        if (nwide) {
            HIPCHK(hipMemcpyAsync(w_g.p, h_wg.data(), nwide * 8, hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(w_x.p, h_wx.data(), nwide * 4, hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(w_q.p, h_wq.data(), nwide * 4, hipMemcpyHostToDevice, s));
        }
        HIPCHK(hipMemcpyAsync(q_n.p, n.data(), nq * 8, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(q_L.p, L.data(), nq * 8, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(q_g0.p, g0.data(), nq * 8, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(q_koff.p, koff.data(), nq * 8, hipMemcpyHostToDevice, s));
        key_off_h = h_key_off;
        if (!h_key_off.empty())
            HIPCHK(hipMemcpyAsync(key_off.p, h_key_off.data(), h_key_off.size() * 4,
                                  hipMemcpyHostToDevice, s));
        for (const KeyedGroup &kg : kgroups) {
            HIPCHK(hipMemcpyAsync(key_x.as<uint32_t>() + kg.g0, kg.kx.data(), kg.kx.size() * 4,
                                  hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(x_m.as<uint64_t>() + kg.g0, kg.km.data(), kg.km.size() * 8,
                                  hipMemcpyHostToDevice, s));
        }
        HIPCHK(hipMemcpyAsync(tile_q.p, t_q.data(), nt * 4, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(tile_x0.p, t_x0.data(), nt * 4, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(tile_nx.p, t_nx.data(), nt * 4, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(tile_g0.p, t_g0.data(), nt * 8, hipMemcpyHostToDevice, s));
        // pageable sources: make sure the copies are done before they go away
        HIPCHK(hipStreamSynchronize(s));

        QueryArgs &q = args;
        q.nq = (uint32_t)nq;
        q.q_n = q_n.as<uint64_t>();
        q.q_L = q_L.as<uint64_t>();
        q.q_g0 = q_g0.as<uint64_t>();
        q.q_koff = q_koff.as<uint64_t>();
        q.key_x = key_x.as<uint32_t>();
        q.key_off = key_off.as<uint32_t>();
        q.x_m = x_m.as<uint64_t>();
        q.x_Y = x_Y.as<uint64_t>();
        q.x_K = x_K.as<uint64_t>();
        q.x_k0 = x_k0.as<uint64_t>();
        q.S = S.as<uint64_t>();
        q.A = A.as<int64_t>();
        q.x_klo = x_klo.as<uint64_t>();
        q.x_khi = x_khi.as<uint64_t>();
        q.ntiles = ntiles;
        q.tile_q = tile_q.as<uint32_t>();
        q.tile_x0 = tile_x0.as<uint32_t>();
        q.tile_nx = tile_nx.as<uint32_t>();
        q.tile_g0 = tile_g0.as<uint64_t>();
        q.tile_ymax = tile_ymax.as<uint64_t>();
        q.tile_klo = tile_klo.as<uint64_t>();
        q.tile_khi = tile_khi.as<uint64_t>();
        q.tile_mode = tile_mode.as<uint32_t>();
        q.tile_nmu = tile_nmu.as<uint32_t>();
        q.tile_items = tile_items.as<uint64_t>();
        q.counter = counter.as<uint32_t>();
        q.pair_stats = pair_stats.as<uint64_t>();
        q.q_nhi = q_nhi.as<uint64_t>();
        q.q_xb = q_xb.as<uint64_t>();
        q.w_n = nwide;
        q.w_g = w_g.as<uint64_t>();
        q.w_x = w_x.as<uint32_t>();
        q.w_q = w_q.as<uint32_t>();
        q.w_mlo = w_mlo.as<uint64_t>();
        q.w_mhi = w_mhi.as<uint64_t>();
        q.w_K = w_K.as<uint64_t>();
        q.w_Y = w_Y.as<uint64_t>();
        q.w_k0 = w_k0.as<uint64_t>();
        q.w_klo = w_klo.as<uint64_t>();
        q.w_khi = w_khi.as<uint64_t>();
        q.beta = t.beta;
        q.ychunk = t.ychunk;
        q.kchunk = t.kchunk;
        q.rl_fast = t.rl_fast;
        q.kbal = t.kbal;
        HIPCHK(launch_zero_u64(pair_stats.as<uint64_t>(), 5, s));
        HIPCHK(launch_plan(q, s));
        HIPCHK(launch_wide_plan(q, s));
        return 0;
    }

    // update prep and item prefix, [event], persistent update
    // band: the tuning whose band applies (nullptr: none, e.g. under graph
    // capture, where b holds no host values of the block)
    int update_block(const BlockArgs &b, uint32_t grid, hipStream_t s, hipEvent_t mid,
                     const Tuning *band = nullptr, hipEvent_t band_ev = nullptr) const
    {
        uint64_t ys = 0, ye = 0;
        const bool use = band && band_of(*band, b.y1, b.y2, ys, ye);
        const uint32_t wa = use ? band->band_lo : 0u, wb = use ? band->band_hi : 0u;
        HIPCHK(launch_update_prep(args, b, s, wa, wb));
        HIPCHK(launch_scan_items(args, s));
        if (mid)
            HIPCHK(hipEventRecord(mid, s));
        HIPCHK(launch_update(args, b, grid, s, wa, wb));
        if (band_ev)  // between the persistent update and the band's kernel
            HIPCHK(hipEventRecord(band_ev, s));
        if (use)
            HIPCHK(launch_ek_window(args, b, ys, ye, s));
        HIPCHK(launch_wide_prep(args, b, s));
        HIPCHK(launch_wide_update(args, b, s));
        return 0;
    }

    // Finalize the listed queries (all when `which` is empty) and gather
    // every A[1] into out_dev.
    int finalize(const std::vector<uint32_t> &which, hipStream_t s)
    {
        if (which.empty()) {
            // keyed groups level by level across the whole grid, plain
            // queries one workgroup each
            std::vector<uint32_t> plain;
            for (uint32_t qi : fin_list) {
                if (koff[qi] == ~0ull) {
                    plain.push_back(qi);
                    continue;
                }
                const uint64_t Lq = L[qi], kbq = koff[qi];
                for (uint64_t hi = Lq, lo = Lq / 2; hi >= 1; hi = lo, lo = lo / 2) {
                    const uint64_t ne = (uint64_t)key_off_h[kbq + hi] - key_off_h[kbq + lo];
                    if (ne == 0)
                        continue;
                    const uint64_t jmax = Lq / (lo + 1);  // terms of the level's smallest x
                    uint32_t gsz = 1;
                    while (gsz < 64 && (uint64_t)gsz * 16 < jmax)
                        gsz *= 2;
                    HIPCHK(launch_finalize_keyed_level(args, qi, lo, hi, ne, gsz, s));
                }
            }
            if (!plain.empty()) {
                HIPCHK(hipMemcpyAsync(qlist.p, plain.data(), plain.size() * 4,
                                      hipMemcpyHostToDevice, s));
                HIPCHK(launch_finalize(args, qlist.as<uint32_t>(), (uint32_t)plain.size(), s));
            }
            HIPCHK(hipStreamSynchronize(s));  // `plain` goes out of scope
        } else {
            HIPCHK(hipMemcpyAsync(qlist.p, which.data(), which.size() * 4, hipMemcpyHostToDevice,
                                  s));
            HIPCHK(launch_finalize(args, qlist.as<uint32_t>(), (uint32_t)which.size(), s));
        }
        HIPCHK(launch_collect(args, out_dev.as<int64_t>(), s));
        return 0;
    }
};

uint32_t update_grid(int ncu, const Tuning &t)
{
    return (uint32_t)std::max(1, ncu * (int)t.waves_per_cu / (UPD_THREADS / 64));
}

uint64_t choose_block(uint64_t req, uint64_t ymax, uint64_t cap = 1ull << 30)
{
    if (req)
        return req;
    const uint64_t need = (ymax / SEG + 1) * SEG;
    return std::min<uint64_t>(need, cap);
}

// ---------------------------------------------------------------------------
// Serving engine
// ---------------------------------------------------------------------------
struct ServeQuery {
    uint64_t n = 0;
    double t_submit = 0, latency = 0;
    int64_t result = 0;
    int state = 0;  // 0 queued, 1 in the sweep, 2 done, 3 failed
    int error = 0;  // state 3: the code its mertens_poll returns
    uint32_t idx = 0;
    uint64_t last_block = 0, seen = 0;
    std::vector<uint8_t> seen_map;
};

struct ServeBatch {
    Batch b;
    std::vector<uint64_t> tickets;
    size_t open = 0;  // queries not yet finalized
    uint64_t x_entries = 0;
};

// One cyclic sweep of the serving worker with the batches riding on it.
struct ServeLane {
    SieveState ss;
    std::vector<std::unique_ptr<ServeBatch>> batches;  // worker thread only
    uint64_t cur_block = 0;
};

struct Server {
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv;
    bool running = false, stop = false;
    int failure = 0;
    hipStream_t stream = nullptr;
    // Lanes by the number of blocks a request needs: lane 0 up to
    // serve_short_blocks (S), lane k up to S 4^k, the last one the rest.
    // Each lane runs its own cyclic sweep over the blocks its requests
    // need, and each worker step runs one block of each busy lane, so a
    // request waits for the cycle of requests of about its own size only.
    static constexpr int NLANES = 6;
    ServeLane lanes[NLANES];
    std::deque<uint64_t> queued;
    std::map<uint64_t, ServeQuery> queries;
    uint64_t next_ticket = 1;
    uint64_t x_used = 0;
    uint64_t blocks_run = 0;
};

constexpr size_t SERVE_CAPACITY_DEFAULT = 4096;
constexpr uint64_t SERVE_X_BUDGET_DEFAULT = 1ull << 26;
constexpr uint64_t SERVE_SHORT_BLOCKS_DEFAULT = 4;

struct Ctx {
    bool ready = false;
    int device = 0;
    int ncu = 256;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t sieve_stream = nullptr;             // sieve-ahead (default priority)
    std::vector<hipEvent_t> sieved_ev, updated_ev;  // per record slot
    uint64_t u_req = 0, block_req = 0;
    Tuning tune;
    size_t serve_capacity = SERVE_CAPACITY_DEFAULT;
    uint64_t serve_x_budget = SERVE_X_BUDGET_DEFAULT;  // x entries in flight (64 B each)
    uint64_t serve_short_blocks = SERVE_SHORT_BLOCKS_DEFAULT;  // requests needing at most this many blocks
    SieveState ss;
    Batch batch;
    DevBuf iv_part, iv_small, iv_vals;  // interval sweep: partial extremes, scalars, values
    // last query (for byproducts): per caller index, L and first global index
    std::vector<uint64_t> last_L, last_g0;
    std::vector<int64_t> last_j;  // index in the batch, -1 for n = 0
    bool last_valid = false;
    double stats[22] = {0};
    hipEvent_t progress_ev = nullptr;
    std::vector<hipEvent_t> events;
    Server srv;
    bool noalloc = false;  // inside mertens_query_noalloc
    bool tuned = false;    // the stored tuning file was applied by mertens_init
};

Ctx g;

// ---------------------------------------------------------------------------
// The no-alloc scratch: one file-scope device array (each device the
// library runs on holds its own copy until the process ends).  Host code
// never uses the name `scratch` as an address: mertens_init takes the
// device address with hipGetSymbolAddress, once per device, and only that
// address reaches kernels and copies.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_SCRATCH_BYTES = 64ull << 20;
constexpr uint64_t NOALLOC_BLOCK = 1ull << 25;  // y per block (16 MiB of records)
constexpr uint64_t NOALLOC_EV_RING = 16;        // blocks of timing events in the ring
static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
uint8_t *g_scratch_dev[MAX_DEVICES] = {nullptr};

// largest interval end: the last block's end and sqrt(b) stay in range
constexpr uint64_t INTERVAL_NMAX = ~0ull - (1ull << 32) + 1;

void serve_stop();

void free_all()
{
    serve_stop();
    g.ss.release();
    g.batch.release();
    g.iv_part.release();
    g.iv_small.release();
    g.iv_vals.release();
    for (hipEvent_t e : g.events)
        (void)hipEventDestroy(e);
    g.events.clear();
    for (hipEvent_t e : g.sieved_ev)
        (void)hipEventDestroy(e);
    for (hipEvent_t e : g.updated_ev)
        (void)hipEventDestroy(e);
    g.sieved_ev.clear();
    g.updated_ev.clear();
    if (g.progress_ev)
        (void)hipEventDestroy(g.progress_ev);
    g.progress_ev = nullptr;
    if (g.sieve_stream)
        (void)hipStreamDestroy(g.sieve_stream);
    g.sieve_stream = nullptr;
    if (g.own_stream)
        (void)hipStreamDestroy(g.own_stream);
    g.own_stream = nullptr;
    g.stream = nullptr;
    g.last_L.clear();
    g.last_g0.clear();
    g.last_j.clear();
    g.last_valid = false;
    g.ready = false;
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

// Record slots for a sweep of nblocks blocks of length B: at most
// sieve_ahead, and at most a quarter of the free device memory.
uint32_t record_slots(uint64_t B, uint64_t nblocks)
{
    size_t free_b = 0, total_b = 0;
    uint64_t cap = g.tune.sieve_ahead;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) {
        const uint64_t have = g.ss.words.bytes;  // already held (reused)
        const uint64_t by_mem = (free_b / 4 + have) / (B / 2);
        cap = std::min<uint64_t>(cap, std::max<uint64_t>(by_mem, 1));
    }
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(cap, nblocks));
}

bool slot_events(uint32_t slots)
{
    while (g.sieved_ev.size() < slots) {
        hipEvent_t a, b;
        if (hipEventCreateWithFlags(&a, hipEventDisableTiming) != hipSuccess)
            return false;
        if (hipEventCreateWithFlags(&b, hipEventDisableTiming) != hipSuccess) {
            (void)hipEventDestroy(a);
            return false;
        }
        g.sieved_ev.push_back(a);
        g.updated_ev.push_back(b);
    }
    return true;
}

// The synchronous sweep for nonzero arguments ns[]: fills A on the device
// and the results into res[] (host).
int run_query(const std::vector<uint64_t> &ns, std::vector<int64_t> &res,
              const std::vector<uint64_t> *ns_hi = nullptr)
{
    const size_t nq = ns.size();
    uint64_t u = g.u_req;
    if (u == 0) {
        long double total = 0;
        if (ns_hi)
            for (size_t i = 0; i < nq; ++i)
                total += (long double)(*ns_hi)[i] * 18446744073709551616.0L + (long double)ns[i];
        else
            total = effective_total_n(ns);
        u = auto_u(total, g.tune.u_scale);
    }
    hipStream_t s = g.stream;
    Batch &bt = g.batch;
    RCCHK(bt.plan(ns, std::vector<uint64_t>(nq, u), g.tune, s, true, ns_hi));
    const uint64_t ymax = bt.ymax_all;
    RCCHK(g.ss.ensure_primes(std::max<uint64_t>(ceil_sqrt_host(ymax), 1024)));
    RCCHK(g.ss.ensure_pattern());
    const uint64_t B = choose_block(g.block_req, ymax, g.tune.block_auto);
    const uint64_t nblocks = ymax / B + 1;
    const uint32_t slots = g.tune.graph ? 1u : record_slots(B, nblocks);
    RCCHK(g.ss.ensure_blocks(B, slots));
    const uint32_t grid = update_grid(g.ncu, g.tune);

    // timing events: [0] start, [1]/[2] around finalize, then six per block
    // in a ring of EV_RING blocks (a block's times are added up before its
    // slot is reused): sieve start and end, prep start, update start, update
    // end, and between the persistent update and the band's kernel
    const uint64_t EV_RING = g.noalloc ? NOALLOC_EV_RING : 4096;
    const uint64_t nring = std::min<uint64_t>(nblocks, EV_RING);
    if (!event_at(3 + 6 * nring) || !slot_events(slots)) {
        set_error_text("hipEventCreate failed");
        return MERTENS_EIO;
    }
    HIPCHK(hipEventRecord(g.events[0], s));
    // one record slot: everything in turn on one stream (no cross-stream
    // waits between the sieve and the update of a block)
    const bool ahead = !g.tune.graph && slots > 1;
    hipStream_t ss = ahead ? g.sieve_stream : s;
    if (ahead)
        HIPCHK(hipStreamWaitEvent(ss, g.events[0], 0));  // after the plan
    RCCHK(g.ss.reset_carry(ss));
    double t_sieve = 0, t_scan = 0, t_prep = 0, t_upd = 0, t_band = 0;
    auto add_times = [&](size_t m) {
        t_sieve += elapsed(m, m + 1);
        t_prep += elapsed(m + 2, m + 3);
        t_upd += elapsed(m + 3, m + 4);
        t_band += elapsed(m + 5, m + 4);
    };
    if (g.tune.graph) {
        // one captured graph of the whole block pipeline, replayed per block;
        // its first node loads the block's parameters from a table
        std::vector<BlockParams> tab(nblocks);
        for (uint64_t bi = 0; bi < nblocks; ++bi)
            tab[bi] = SieveState::params_of(
                g.ss.make_block(bi * B, std::min(bi * B + B - 1, ymax)));
        RCCHK(ensure(g.ss.bp_table, nblocks * sizeof(BlockParams)));
        HIPCHK(hipMemcpyAsync(g.ss.bp_table.p, tab.data(), nblocks * sizeof(BlockParams),
                              hipMemcpyHostToDevice, s));
        HIPCHK(launch_zero_u64(g.ss.bp_index.as<uint64_t>(), 1, s));
        HIPCHK(hipStreamSynchronize(s));  // the host table goes out of scope
        const BlockArgs bm = g.ss.max_block(B);
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        int rc = 0;
        if (launch_block_next(g.ss.bp_table.as<BlockParams>(), g.ss.bp_cur.as<BlockParams>(),
                              g.ss.bp_index.as<uint32_t>(), s) != hipSuccess)
            rc = MERTENS_EIO;
        if (!rc)
            rc = g.ss.sieve(bm, s, nullptr, false);
        if (!rc)
            rc = bt.update_block(bm, grid, s, nullptr);
        const hipError_t ec = hipStreamEndCapture(s, &graph);
        if (rc || ec != hipSuccess) {
            if (graph)
                (void)hipGraphDestroy(graph);
            if (rc)
                return rc;
            HIPCHK(ec);
        }
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(graph);
            HIPCHK(ei);
        }
        hipError_t el = hipSuccess;
        for (uint64_t bi = 0; bi < nblocks && el == hipSuccess; ++bi)
            el = hipGraphLaunch(exec, s);
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        HIPCHK(el);
    }
    // Direct launches: the sieve runs ahead on its own stream into a ring of
    // record slots, so blocks b+1, b+2, ... are sieved while block b is
    // updated (block 0 holds most of the update work).  Block b waits for
    // its sieve; the sieve of block b reuses the slot of block b - slots
    // once that block's update is done.  The carry between blocks stays in
    // sieve order on the sieve stream.
    for (uint64_t bi = 0; bi < nblocks && !g.tune.graph; ++bi) {
        const uint64_t y1 = bi * B;
        const uint64_t y2 = std::min(y1 + B - 1, ymax);
        const uint32_t slot = (uint32_t)(bi % slots);
        const BlockArgs b = g.ss.make_block(y1, y2, slot);
        const size_t ev = 3 + 6 * (size_t)(bi % EV_RING);
        if (bi >= EV_RING) {  // the slot's previous block: wait for it, keep its times
            HIPCHK(hipEventSynchronize(g.events[ev + 4]));
            add_times(ev);
        }
        if (ahead && bi >= slots)
            HIPCHK(hipStreamWaitEvent(ss, g.updated_ev[slot], 0));
        RCCHK(g.ss.sieve(b, ss, g.events[ev]));
        HIPCHK(hipEventRecord(g.events[ev + 1], ss));
        if (ahead) {
            HIPCHK(hipEventRecord(g.sieved_ev[slot], ss));
            HIPCHK(hipStreamWaitEvent(s, g.sieved_ev[slot], 0));
        }
        HIPCHK(hipEventRecord(g.events[ev + 2], s));
        const uint64_t W = g.tune.update_window ? (1ull << g.tune.update_window) : 0;
        if (W && y1 < g.tune.window_ymax && y2 - y1 >= W &&
            (y2 - y1) / W < SieveState::MAX_WINDOWS) {
            uint32_t w = 0;
            const uint64_t nw = (y2 - y1) / W + 1;
            for (uint64_t ua = y1; ua <= y2; ua += W, ++w) {
                const BlockArgs bw = g.ss.window_of(b, ua, std::min(ua + W - 1, y2), w);
                HIPCHK(launch_block_set(SieveState::params_of(bw),
                                        const_cast<BlockParams *>(bw.bp), s));
                RCCHK(bt.update_block(bw, grid, s, w == 0 ? g.events[ev + 3] : nullptr, &g.tune,
                                      w + 1 == nw ? g.events[ev + 5] : nullptr));
                if (g.tune.progress) {  // windows of a heavy block report one by one
                    if (!g.progress_ev)
                        HIPCHK(hipEventCreateWithFlags(&g.progress_ev, hipEventDisableTiming));
                    HIPCHK(hipEventRecord(g.progress_ev, s));
                    HIPCHK(hipEventSynchronize(g.progress_ev));
                    fprintf(stderr, "mertens: block %llu window %u of %llu updated\n",
                            (unsigned long long)bi, w + 1, (unsigned long long)nw);
                    fflush(stderr);
                }
            }
        } else {
            RCCHK(bt.update_block(b, grid, s, g.events[ev + 3], &g.tune, g.events[ev + 5]));
        }
        HIPCHK(hipEventRecord(g.events[ev + 4], s));
        if (ahead)
            HIPCHK(hipEventRecord(g.updated_ev[slot], s));
        if (g.tune.progress && (bi + 1) % g.tune.progress == 0) {
            HIPCHK(hipEventSynchronize(g.events[ev + 4]));
            fprintf(stderr, "mertens: block %llu of %llu updated\n", (unsigned long long)(bi + 1),
                    (unsigned long long)nblocks);
            fflush(stderr);
        }
    }
    HIPCHK(hipEventRecord(g.events[1], s));
    RCCHK(bt.finalize({}, s));
    HIPCHK(hipEventRecord(g.events[2], s));
    res.resize(nq);
    uint64_t pst[5] = {0, 0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(res.data(), bt.out_dev.p, nq * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(pst, bt.pair_stats.p, 40, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (ahead)
        HIPCHK(hipStreamSynchronize(ss));

    // kernel times per stream; with sieve-ahead they overlap, so their sum
    // can exceed the total
    if (!g.tune.graph)
        for (uint64_t bj = nblocks - nring; bj < nblocks; ++bj)
            add_times(3 + 6 * (size_t)(bj % EV_RING));
    g.stats[0] = (double)(ymax + 1);
    g.stats[1] = (double)nblocks;
    g.stats[2] = (double)u;
    g.stats[3] = (double)bt.X;
    g.stats[4] = (double)pst[0];
    g.stats[5] = (double)pst[1];
    g.stats[6] = t_sieve;
    g.stats[7] = t_scan;
    g.stats[8] = t_prep;
    g.stats[9] = t_upd;
    g.stats[10] = elapsed(1, 2);
    g.stats[11] = elapsed(0, 2);
    g.stats[12] = (double)nblocks;
    g.stats[13] = (double)nblocks;
    g.stats[14] = (double)pst[2];
    g.stats[15] = (double)pst[3];
    g.stats[20] = t_band;
    g.stats[21] = (double)pst[4];
    for (int i = 16; i < 20; ++i)
        g.stats[i] = 0;
    return 0;
}

// ---------------------------------------------------------------------------
// Serving worker
// ---------------------------------------------------------------------------
void serve_fail(int rc)
{
    Server &v = g.srv;
    std::lock_guard<std::mutex> lk(v.mu);
    v.failure = rc;
    for (auto &kv : v.queries)
        if (kv.second.state < 2)
            kv.second.state = 3;
    v.queued.clear();
}

// The lane of a request (or batch) that needs `blocks` blocks.
int serve_lane_of(uint64_t blocks)
{
    uint64_t lim = std::max<uint64_t>(g.serve_short_blocks, 1);
    int k = 0;
    while (k < Server::NLANES - 1 && blocks > lim) {
        lim *= 4;
        ++k;
    }
    return k;
}

// Plan the admitted tickets as one batch and put it on the lane its
// longest request needs.
int serve_admit(const std::vector<uint64_t> &tickets, uint64_t B)
{
    Server &v = g.srv;
    hipStream_t s = v.stream;
    auto sb = std::make_unique<ServeBatch>();
    std::vector<uint64_t> ns, us;
    {
        std::lock_guard<std::mutex> lk(v.mu);
        for (uint64_t t : tickets)
            ns.push_back(v.queries[t].n);
    }
    // the requests admitted together share one split u, as one query call
    // does (u ~ (sum of their n)^(2/3)): the update work, ~ (sum of n) /
    // sqrt(u), then falls, the sweep grows by much less
    const uint64_t u_shared = g.u_req ? g.u_req : auto_u(effective_total_n(ns), g.tune.u_scale);
    us.assign(ns.size(), u_shared);
    // no keyed groups here: requests complete and finalize one by one
    RCCHK(sb->b.plan(ns, us, g.tune, s, false));
    sb->tickets = tickets;
    sb->open = tickets.size();
    sb->x_entries = sb->b.X;
    uint64_t maxlb = 0;
    {
        std::lock_guard<std::mutex> lk(v.mu);
        // admission reserved each request's entries at its own u; the batch
        // holds b.X entries at the shared u (never more)
        uint64_t reserved = 0;
        for (uint64_t x : ns)
            reserved += std::max<uint64_t>(1, x / (g.u_req ? g.u_req : auto_u((long double)x,
                                                                              g.tune.u_scale)));
        v.x_used = v.x_used - std::min(v.x_used, reserved) + sb->b.X;
        for (size_t i = 0; i < tickets.size(); ++i) {
            ServeQuery &q = v.queries[tickets[i]];
            q.state = 1;
            q.idx = (uint32_t)i;
            q.last_block = sb->b.ymax[i] / B;
            q.seen = 0;
            q.seen_map.assign(q.last_block + 1, 0);
            maxlb = std::max(maxlb, q.last_block);
        }
    }
    v.lanes[serve_lane_of(maxlb + 1)].batches.push_back(std::move(sb));
    return 0;
}

// One block of lane ln's cyclic sweep for every batch on it; finalize the
// queries that have now seen every block they need.
int serve_lane_step(ServeLane &ln, uint64_t B)
{
    Server &v = g.srv;
    hipStream_t s = v.stream;
    if (ln.batches.empty())
        return 0;
    // pass length: every block some query in flight on the lane still needs
    uint64_t ymax = 0;
    {
        std::lock_guard<std::mutex> lk(v.mu);
        for (auto &sb : ln.batches)
            for (size_t i = 0; i < sb->tickets.size(); ++i)
                if (v.queries[sb->tickets[i]].state == 1)
                    ymax = std::max(ymax, sb->b.ymax[i]);
    }
    const uint64_t nb = ymax / B + 1;
    if (ln.cur_block >= nb)
        ln.cur_block = 0;
    // Blocks are always sieved whole: the pass may grow while it runs, and
    // the carry into the next block must then cover the whole block.
    RCCHK(ln.ss.ensure_primes(std::max<uint64_t>(ceil_sqrt_host(nb * B), 1024)));
    RCCHK(ln.ss.ensure_pattern());
    RCCHK(ln.ss.ensure_blocks(B));
    if (ln.cur_block == 0)
        RCCHK(ln.ss.reset_carry(s));
    const uint64_t y1 = ln.cur_block * B;
    const uint64_t y2 = y1 + B - 1;
    const BlockArgs b = ln.ss.make_block(y1, y2);
    RCCHK(ln.ss.sieve(b, s, nullptr));
    const uint32_t grid = update_grid(g.ncu, g.tune);
    for (auto &sb : ln.batches)
        if (sb->open)
            RCCHK(sb->b.update_block(b, grid, s, nullptr, &g.tune));

    // bookkeeping: which queries have now seen every block they need
    std::vector<std::pair<ServeBatch *, std::vector<uint32_t>>> done;
    {
        std::lock_guard<std::mutex> lk(v.mu);
        for (auto &sb : ln.batches) {
            std::vector<uint32_t> fin;
            for (size_t i = 0; i < sb->tickets.size(); ++i) {
                ServeQuery &q = v.queries[sb->tickets[i]];
                if (q.state != 1)
                    continue;
                if (ln.cur_block <= q.last_block && !q.seen_map[ln.cur_block]) {
                    q.seen_map[ln.cur_block] = 1;
                    q.seen++;
                }
                if (q.seen == q.last_block + 1)
                    fin.push_back((uint32_t)i);
            }
            if (!fin.empty())
                done.emplace_back(sb.get(), fin);
        }
    }
    ln.cur_block++;
    v.blocks_run++;
    for (auto &d : done) {
        ServeBatch *sb = d.first;
        RCCHK(sb->b.finalize(d.second, s));
        std::vector<int64_t> out(sb->tickets.size());
        HIPCHK(hipMemcpyAsync(out.data(), sb->b.out_dev.p, out.size() * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double t = now_s();
        std::lock_guard<std::mutex> lk(v.mu);
        for (uint32_t i : d.second) {
            ServeQuery &q = v.queries[sb->tickets[i]];
            q.result = out[i];
            q.latency = t - q.t_submit;
            q.state = 2;
            sb->open--;
        }
    }
    // retire batches whose queries are all finalized
    {
        std::lock_guard<std::mutex> lk(v.mu);
        for (auto it = ln.batches.begin(); it != ln.batches.end();) {
            if ((*it)->open == 0) {
                v.x_used -= (*it)->x_entries;
                (*it)->b.release();
                it = ln.batches.erase(it);
            } else {
                ++it;
            }
        }
    }
    return 0;
}

// One worker step: admit queued requests (split by lane), then one block of
// each busy lane.
int serve_step(std::vector<uint64_t> &admit)
{
    Server &v = g.srv;
    const uint64_t B = g.block_req ? g.block_req : (1ull << 30);
    if (!admit.empty()) {
        std::vector<uint64_t> by_lane[Server::NLANES];
        for (uint64_t t : admit) {
            uint64_t n;
            {
                std::lock_guard<std::mutex> lk(v.mu);
                n = v.queries[t].n;
            }
            const uint64_t u = g.u_req ? g.u_req : auto_u((long double)n, g.tune.u_scale);
            const uint64_t L = std::max<uint64_t>(1, n / u);
            by_lane[serve_lane_of((n / (L + 1)) / B + 1)].push_back(t);
        }
        for (auto &tl : by_lane) {
            if (tl.empty())
                continue;
            const int rc = serve_admit(tl, B);
            if (rc != 0) {
                // only this batch fails: its tickets report rc, their x
                // entries return to the budget, and the sweep goes on
                std::lock_guard<std::mutex> lk(v.mu);
                for (uint64_t t : tl) {
                    ServeQuery &q = v.queries[t];
                    const uint64_t u = g.u_req ? g.u_req : auto_u((long double)q.n, g.tune.u_scale);
                    const uint64_t need = std::max<uint64_t>(1, q.n / u);
                    v.x_used -= std::min(v.x_used, need);
                    q.state = 3;
                    q.error = rc;
                }
            }
        }
    }
    for (ServeLane &ln : v.lanes)
        RCCHK(serve_lane_step(ln, B));
    v.cv.notify_all();
    return 0;
}

void serve_loop()
{
    Server &v = g.srv;
    if (hipSetDevice(g.device) != hipSuccess) {
        serve_fail(MERTENS_EIO);
        return;
    }
    for (;;) {
        std::vector<uint64_t> admit;
        {
            std::unique_lock<std::mutex> lk(v.mu);
            v.cv.wait(lk, [&] {
                bool busy = false;
                for (const ServeLane &ln : v.lanes)
                    busy = busy || !ln.batches.empty();
                return v.stop || !v.queued.empty() || busy;
            });
            if (v.stop)
                break;
            // admission by device memory: x entries in flight stay within budget
            while (!v.queued.empty()) {
                ServeQuery &q = v.queries[v.queued.front()];
                const uint64_t u = g.u_req ? g.u_req : auto_u((long double)q.n, g.tune.u_scale);
                const uint64_t need = std::max<uint64_t>(1, q.n / u);
                if (v.x_used > 0 && v.x_used + need > g.serve_x_budget)
                    break;
                v.x_used += need;
                admit.push_back(v.queued.front());
                v.queued.pop_front();
            }
        }
        const int rc = serve_step(admit);
        if (rc != 0) {
            serve_fail(rc);
            std::unique_lock<std::mutex> lk(v.mu);
            v.cv.notify_all();
            v.cv.wait(lk, [&] { return v.stop; });
            break;
        }
    }
    std::lock_guard<std::mutex> lk(v.mu);
    for (ServeLane &ln : v.lanes) {
        for (auto &sb : ln.batches)
            sb->b.release();
        ln.batches.clear();
    }
}

int serve_start()
{
    Server &v = g.srv;
    if (v.running)
        return 0;
    HIPCHK(hipStreamCreateWithFlags(&v.stream, hipStreamNonBlocking));
    v.stop = false;
    v.failure = 0;
    for (ServeLane &ln : v.lanes)
        ln.cur_block = 0;
    v.x_used = 0;
    v.running = true;
    v.worker = std::thread(serve_loop);
    return 0;
}

void serve_stop()
{
    Server &v = g.srv;
    if (!v.running)
        return;
    {
        std::lock_guard<std::mutex> lk(v.mu);
        v.stop = true;
    }
    v.cv.notify_all();
    v.worker.join();
    (void)hipStreamSynchronize(v.stream);
    (void)hipStreamDestroy(v.stream);
    v.stream = nullptr;
    for (ServeLane &ln : v.lanes)
        ln.ss.release();
    v.queries.clear();
    v.queued.clear();
    v.running = false;
}

}  // namespace

// ======================================================================
// C ABI
// ======================================================================
extern "C" {

// The autotuner's choice: tuned_<arch>.json next to this library, applied
// when its "source_sha256" equals the hash of the kernel sources compiled
// in (a file measured on other kernels is ignored); MERTENS_TUNED=0 skips
// it.  Only the flat "params" object is read ("key": number pairs), each
// through mertens_set_param (a value it refuses is skipped).
static void load_tuned()
{
    g.tuned = false;
    const char *env = getenv("MERTENS_TUNED");
    if ((env && !strcmp(env, "0")) || !MERTENS_KERNEL_SHA256[0])
        return;
    Dl_info info;
    if (!dladdr(reinterpret_cast<void *>(&mertens_init), &info) || !info.dli_fname)
        return;
    std::string path(info.dli_fname);
    path = path.substr(0, path.rfind('/') + 1) + "tuned_" MERTENS_ARCH_NAME ".json";
    FILE *f = fopen(path.c_str(), "rb");
    if (!f)
        return;
    std::string txt;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0 && txt.size() < (1u << 20))
        txt.append(buf, got);
    fclose(f);
    auto string_after = [&](const char *key, size_t from, size_t &end) -> std::string {
        const size_t k = txt.find(key, from);
        if (k == std::string::npos)
            return std::string();
        const size_t a = txt.find('"', txt.find(':', k + strlen(key)) + 1);
        const size_t b = a == std::string::npos ? a : txt.find('"', a + 1);
        if (b == std::string::npos)
            return std::string();
        end = b + 1;
        return txt.substr(a + 1, b - a - 1);
    };
    size_t pos = 0;
    if (string_after("\"source_sha256\"", 0, pos) != MERTENS_KERNEL_SHA256)
        return;
    size_t p = txt.find("\"params\"");
    p = p == std::string::npos ? p : txt.find('{', p);
    if (p == std::string::npos)
        return;
    ++p;
    for (;;) {
        const size_t a = txt.find_first_not_of(" \t\r\n,", p);
        if (a == std::string::npos || txt[a] != '"')
            break;
        const size_t b = txt.find('"', a + 1);
        const size_t c = b == std::string::npos ? b : txt.find(':', b);
        if (c == std::string::npos)
            break;
        const std::string key = txt.substr(a + 1, b - a - 1);
        char *endp = nullptr;
        const double v = strtod(txt.c_str() + c + 1, &endp);
        if (endp == txt.c_str() + c + 1)
            break;
        (void)mertens_set_param(key.c_str(), v);
        p = (size_t)(endp - txt.c_str());
    }
    g.tuned = true;
}

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
    HIPCHK(hipStreamCreateWithFlags(&g.sieve_stream, hipStreamNonBlocking));
    g.stream = g.own_stream;
    g.u_req = u;
    g.block_req = block;
    g.tune = Tuning();
    g.ss.bucket_min = SieveState().bucket_min;
    g.serve_capacity = SERVE_CAPACITY_DEFAULT;
    g.serve_x_budget = SERVE_X_BUDGET_DEFAULT;
    g.serve_short_blocks = SERVE_SHORT_BLOCKS_DEFAULT;
    load_tuned();
    int rc = g.ss.ensure_pattern();
    if (rc == 0)
        rc = g.ss.ensure_primes(1024);
    // the no-alloc scratch of this device (its address, once per device)
    // and the timing events a no-alloc call uses, created here
    if (rc == 0 && g.device >= 0 && g.device < MAX_DEVICES && !g_scratch_dev[g.device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error("hipGetSymbolAddress(scratch)", e, __FILE__, __LINE__);
            rc = MERTENS_EIO;
        } else {
            g_scratch_dev[g.device] = static_cast<uint8_t *>(ptr);
        }
    }
    if (rc == 0 && (!event_at(3 + 6 * NOALLOC_EV_RING) || !slot_events(1))) {
        set_error_text("hipEventCreate failed");
        rc = MERTENS_EIO;
    }
    if (rc != 0) {
        free_all();
        return rc;
    }
    g.ready = true;
    return 0;
}

int mertens_query_noalloc(const uint64_t *n, size_t count, int64_t *out)
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
    if (g.srv.running) {
        set_error_text("mertens_query_noalloc cannot run beside the serving worker");
        return MERTENS_EINVAL;
    }
    uint8_t *base = (g.device >= 0 && g.device < MAX_DEVICES) ? g_scratch_dev[g.device] : nullptr;
    if (!base) {
        set_error_text("no no-alloc scratch on this device");
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
    int rc = 0;
    if (!ns.empty()) {
        // a fresh sieve state and batch whose every buffer is a piece of the
        // scratch; the library's own state is put back afterwards
        SieveState ss_mine;
        ss_mine.bucket_min = g.ss.bucket_min;
        Batch bt_mine;
        std::swap(g.ss, ss_mine);
        std::swap(g.batch, bt_mine);
        const Tuning saved = g.tune;
        const uint64_t saved_block = g.block_req;
        g.tune.graph = false;
        g.tune.sieve_ahead = 1;
        g.tune.progress = 0;
        g.tune.update_window = 0;
        if (!g.block_req || g.block_req > NOALLOC_BLOCK)
            g.block_req = NOALLOC_BLOCK;
        g.noalloc = true;
        g_arena = Arena{base, NOALLOC_SCRATCH_BYTES, 0, true};
        rc = g.ss.copy_pattern(ss_mine.pattern, g.stream);
        if (rc == 0)
            rc = run_query(ns, res);
        // nothing of this call may still run when the next one reuses the scratch
        const hipError_t e1 = hipStreamSynchronize(g.stream);
        const hipError_t e2 = hipStreamSynchronize(g.sieve_stream);
        if (rc == 0 && (e1 != hipSuccess || e2 != hipSuccess)) {
            set_error("hipStreamSynchronize", e1 != hipSuccess ? e1 : e2, __FILE__, __LINE__);
            rc = MERTENS_EIO;
        }
        g_arena.on = false;
        g.noalloc = false;
        g.tune = saved;
        g.block_req = saved_block;
        std::swap(g.ss, ss_mine);
        std::swap(g.batch, bt_mine);
        ss_mine.release();  // scratch pieces only: nothing is freed
        bt_mine.release();
    }
    if (rc != 0)
        return rc;
    for (size_t i = 0; i < count; ++i)
        out[i] = 0;
    for (size_t j = 0; j < where.size(); ++j)
        out[where[j]] = res[j];
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
    g.last_valid = false;
    if (!ns.empty()) {
        int rc = run_query(ns, res);
        if (rc != 0)
            return rc;
    }
    g.last_L.assign(count, 0);
    g.last_g0.assign(count, 0);
    g.last_j.assign(count, -1);
    for (size_t i = 0; i < count; ++i)
        out[i] = 0;
    for (size_t j = 0; j < where.size(); ++j) {
        out[where[j]] = res[j];
        g.last_L[where[j]] = g.batch.L[j];
        g.last_g0[where[j]] = g.batch.g0[j];
        g.last_j[where[j]] = (int64_t)j;
    }
    g.last_valid = true;
    return 0;
}

int mertens_query_wide(const uint64_t *n_lo, const uint64_t *n_hi, size_t count, int64_t *out)
{
    if (count == 0)
        return 0;
    if (!n_lo || !n_hi || !out) {
        set_error_text("null pointer with count > 0");
        return MERTENS_EINVAL;
    }
    for (size_t i = 0; i < count; ++i)
        if (n_hi[i] >> 32) {
            set_error_text("wide arguments must be below 2^96");
            return MERTENS_EINVAL;
        }
    if (!g.ready) {
        set_error_text("mertens_init has not been called");
        return MERTENS_ENODEV;
    }
    std::vector<uint64_t> lo, hi;
    std::vector<size_t> where;
    for (size_t i = 0; i < count; ++i)
        if (n_lo[i] != 0 || n_hi[i] != 0) {
            lo.push_back(n_lo[i]);
            hi.push_back(n_hi[i]);
            where.push_back(i);
        }
    std::vector<int64_t> res;
    g.last_valid = false;
    if (!lo.empty()) {
        int rc = run_query(lo, res, &hi);
        if (rc != 0)
            return rc;
    }
    g.last_L.assign(count, 0);
    g.last_g0.assign(count, 0);
    g.last_j.assign(count, -1);
    for (size_t i = 0; i < count; ++i)
        out[i] = 0;
    for (size_t j = 0; j < where.size(); ++j) {
        out[where[j]] = res[j];
        g.last_L[where[j]] = g.batch.L[j];
        g.last_g0[where[j]] = g.batch.g0[j];
        g.last_j[where[j]] = (int64_t)j;
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
    if (k == 0)
        return 0;
    const int64_t j = g.last_j[i];
    if (j >= 0 && g.batch.koff[(size_t)j] != ~0ull) {
        // member of a keyed group: gather its entries (c, floor(n/c))
        RCCHK(ensure(g.batch.byp, k * 8));
        HIPCHK(launch_keyed_byproducts(g.batch.args, (uint32_t)j, k, g.batch.byp.as<int64_t>(),
                                       g.stream));
        HIPCHK(hipMemcpyAsync(buf, g.batch.byp.p, k * 8, hipMemcpyDeviceToHost, g.stream));
    } else {
        HIPCHK(hipMemcpyAsync(buf, g.batch.A.as<int64_t>() + g.last_g0[i], k * 8,
                              hipMemcpyDeviceToHost, g.stream));
    }
    HIPCHK(hipStreamSynchronize(g.stream));
    return 0;
}

int mertens_interval(uint64_t a, uint64_t b, const int64_t *m_a, int64_t *m_b, uint64_t *n_ext,
                     int64_t *m_ext, int64_t *values, size_t cap)
{
    if (a == 0 || b < a || b > INTERVAL_NMAX) {
        set_error_text("interval needs 1 <= a <= b <= 2^64 - 2^32");
        return MERTENS_EINVAL;
    }
    const uint64_t len = b - a + 1;  // no wrap: b - a < 2^64 - 1
    if (values && (len > (1ull << 28) || cap < len)) {
        set_error_text("values needs cap >= b - a + 1 and b - a + 1 <= 2^28");
        return MERTENS_EINVAL;
    }
    if (!g.ready) {
        set_error_text("mertens_init has not been called");
        return MERTENS_ENODEV;
    }
    int64_t ma = 0;
    if (m_a) {
        ma = *m_a;
    } else {
        std::vector<int64_t> r;
        g.last_valid = false;  // the query replaces the last query's arrays
        RCCHK(run_query({a}, r));
        ma = r[0];
    }
    hipStream_t s = g.stream;
    const uint64_t start = a - a % SEG;
    RCCHK(g.ss.ensure_primes(std::max<uint64_t>(ceil_sqrt_host(b), 1024)));
    RCCHK(g.ss.ensure_pattern());
    // automatic blocks of up to 2^31 y: at high offsets every block visits every
    // sieving prime (residues, buckets), so longer blocks cost less per value
    const uint64_t B =
        g.block_req ? g.block_req : std::min<uint64_t>((b - start) / SEG * SEG + SEG, 1ull << 31);
    RCCHK(g.ss.ensure_blocks(B, 1));
    RCCHK(ensure(g.iv_part, (size_t)IV_WGS * 32));
    RCCHK(ensure(g.iv_small, 64));  // off at [0], results at [1..5]
    if (values)
        RCCHK(ensure(g.iv_vals, len * 8));
    const uint64_t nblocks = (b - start) / B + 1;
    // timing events: [0] start, [1] end, then seven per block in a ring of
    // EV_RING blocks (a block's times are added up before its slot is reused)
    const uint64_t EV_RING = g.noalloc ? NOALLOC_EV_RING : 4096;
    const uint64_t nring = std::min<uint64_t>(nblocks, EV_RING);
    if (!event_at(2 + 7 * nring)) {
        set_error_text("hipEventCreate failed");
        return MERTENS_EIO;
    }
    int64_t *off = g.iv_small.as<int64_t>(), *res = off + 1;
    HIPCHK(hipEventRecord(g.events[0], s));
    RCCHK(g.ss.reset_carry(s));
    HIPCHK(launch_zero_u64(g.iv_part.as<uint64_t>(), (size_t)IV_WGS * 4, s));
    uint64_t *bk_total = reinterpret_cast<uint64_t *>(g.ss.carry.as<uint8_t>() + 16);
    HIPCHK(launch_zero_u64(bk_total, 1, s));
    double t_sieve = 0, t_prep = 0, t_red = 0, t_fill = 0, t_regroup = 0;
    std::vector<uint8_t> filled(nring, 0);  // per ring slot: its block used buckets
    auto add_times = [&](uint64_t bj) {
        const size_t m = 2 + 7 * (size_t)(bj % EV_RING);
        t_prep += elapsed(m, m + 3);
        t_sieve += elapsed(m + 3, m + 1);
        t_red += elapsed(m + 1, m + 2);
        if (filled[bj % EV_RING]) {
            t_fill += elapsed(m + 4, m + 5);
            t_regroup += elapsed(m + 5, m + 6);
        }
    };
    double bucket_primes = 0;
    uint64_t bi = 0;
    for (uint64_t y1 = start;; y1 += B, ++bi) {
        const uint64_t y2 = b - y1 < B ? b : y1 + B - 1;
        const BlockArgs blk = g.ss.make_block(y1, y2);
        bucket_primes += (double)(blk.n_sieve - blk.n_bucket);
        const size_t ev = 2 + 7 * (size_t)(bi % EV_RING);
        if (bi >= EV_RING) {  // the slot's previous block: wait for it, keep its times
            HIPCHK(hipEventSynchronize(g.events[ev + 2]));
            add_times(bi - EV_RING);
        }
        filled[bi % EV_RING] = blk.n_bucket < blk.n_sieve;
        HIPCHK(hipEventRecord(g.events[ev], s));
        RCCHK(g.ss.sieve(blk, s, g.events[ev + 3], true, g.events[ev + 4], g.events[ev + 5],
                         g.events[ev + 6]));
        HIPCHK(hipEventRecord(g.events[ev + 1], s));
        if (y1 == start)
            HIPCHK(launch_interval_base(blk, a, ma, off, s));
        const uint64_t lo = std::max(y1, a);
        HIPCHK(launch_interval_extreme(blk, lo, y2, off, g.iv_part.as<uint64_t>(), s));
        if (values)
            HIPCHK(launch_interval_values(blk, lo, y2 - lo + 1, off,
                                          g.iv_vals.as<int64_t>() + (lo - a), s));
        if (y2 == b)
            HIPCHK(launch_interval_final(blk, g.iv_part.as<uint64_t>(), b, off, res, s));
        HIPCHK(hipEventRecord(g.events[ev + 2], s));
        if (y2 == b)
            break;
    }
    HIPCHK(hipEventRecord(g.events[1], s));
    int64_t h[5];
    uint64_t entries = 0;
    HIPCHK(hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&entries, bk_total, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (values)
        HIPCHK(hipMemcpy(values, g.iv_vals.p, len * 8, hipMemcpyDeviceToHost));
    if (m_b)
        *m_b = h[4];
    if (n_ext) {
        n_ext[0] = (uint64_t)h[0];
        n_ext[1] = (uint64_t)h[2];
    }
    if (m_ext) {
        m_ext[0] = h[1];
        m_ext[1] = h[3];
    }
    for (uint64_t bj = nblocks - nring; bj < nblocks; ++bj)
        add_times(bj);
    for (double &v : g.stats)
        v = 0;
    g.stats[0] = (double)(b - start + 1);
    g.stats[1] = (double)nblocks;
    g.stats[6] = t_sieve;
    g.stats[8] = t_prep;
    g.stats[9] = t_red;
    g.stats[11] = elapsed(0, 1);
    g.stats[13] = (double)nblocks;
    g.stats[16] = (double)entries;
    g.stats[17] = t_fill;
    g.stats[18] = bucket_primes;
    g.stats[19] = t_regroup;
    return 0;
}

int mertens_submit(uint64_t n, uint64_t *ticket)
{
    if (!ticket)
        return MERTENS_EINVAL;
    if (!g.ready)
        return MERTENS_ENODEV;
    // the request's own split must give a plan (as Batch::plan requires)
    if (n > 0) {
        const uint64_t u = g.u_req ? g.u_req : auto_u((long double)n, g.tune.u_scale);
        const uint64_t Lw = n / u;
        if (Lw >= (1ull << 31)) {
            set_error_text("u too small for this n: its array would need 2^31 or more entries");
            return MERTENS_EINVAL;
        }
        if ((n / ((Lw < 1 ? 1 : Lw) + 1)) >> 62) {
            set_error_text("u too large for this n: the sieve bound n/(L+1) must stay below 2^62");
            return MERTENS_EINVAL;
        }
    }
    Server &v = g.srv;
    if (!v.running)
        RCCHK(serve_start());
    std::lock_guard<std::mutex> lk(v.mu);
    if (v.failure)
        return v.failure;
    size_t inflight = 0;
    for (auto &kv : v.queries)
        inflight += kv.second.state < 2;
    if (inflight >= g.serve_capacity)
        return MERTENS_EAGAIN;
    const uint64_t t = v.next_ticket++;
    ServeQuery &q = v.queries[t];
    q.n = n;
    q.t_submit = now_s();
    if (n == 0) {
        q.state = 2;  // M(0) = 0, nothing to compute
        q.result = 0;
    } else {
        v.queued.push_back(t);
    }
    *ticket = t;
    v.cv.notify_all();
    return 0;
}

int mertens_poll(uint64_t ticket, int64_t *out, double *latency_s)
{
    if (!g.ready)
        return MERTENS_ENODEV;
    Server &v = g.srv;
    std::lock_guard<std::mutex> lk(v.mu);
    auto it = v.queries.find(ticket);
    if (it == v.queries.end())
        return MERTENS_ERANGE;
    ServeQuery &q = it->second;
    if (q.state == 3) {
        const int rc = q.error ? q.error : (v.failure ? v.failure : MERTENS_EIO);
        v.queries.erase(it);
        return rc;
    }
    if (q.state != 2)
        return MERTENS_EINPROGRESS;
    if (out)
        *out = q.result;
    if (latency_s)
        *latency_s = (q.n == 0) ? 0.0 : q.latency;
    v.queries.erase(it);
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
    if (g.srv.running && strncmp(key, "serve_", 6) != 0) {
        set_error_text("tuning parameters cannot change while serving");
        return MERTENS_EINVAL;
    }
    if (!strcmp(key, "u_scale")) {
        if (!(value >= 1e-3 && value <= 1e3))
            return MERTENS_EINVAL;
        g.tune.u_scale = value;
    } else if (!strcmp(key, "graph")) {
        if (!(value == 0.0 || value == 1.0))
            return MERTENS_EINVAL;
        g.tune.graph = value != 0.0;
    } else if (!strcmp(key, "progress")) {
        if (!(value >= 0.0 && value <= 1e12 && value == std::floor(value)))
            return MERTENS_EINVAL;
        g.tune.progress = (uint64_t)value;
    } else if (!strcmp(key, "wide_bits")) {
        if (!(value >= 33.0 && value <= 64.0 && value == std::floor(value)))
            return MERTENS_EINVAL;
        g.tune.wide_bits = (uint32_t)value;
    } else if (!strcmp(key, "beta")) {
        if (!(value > 0.0 && value <= 1.0))
            return MERTENS_EINVAL;
        g.tune.beta = value;
    } else if (!strcmp(key, "ychunk")) {
        // partial sums of a work item stay below ychunk * 2^32 <= 2^52: exact in fp64
        if (!(value >= 64 && value <= (1 << 20)) || ((uint64_t)value) % 64 != 0)
            return MERTENS_EINVAL;
        g.tune.ychunk = (uint32_t)value;
    } else if (!strcmp(key, "kchunk")) {
        if (!(value >= 64 && value <= (1 << 24)))
            return MERTENS_EINVAL;
        g.tune.kchunk = (uint32_t)value;
    } else if (!strcmp(key, "kbal")) {
        if (!(value >= 0 && value <= 1024) || value != (double)(int)value)
            return MERTENS_EINVAL;
        g.tune.kbal = (uint32_t)value;
    } else if (!strcmp(key, "bucket_min")) {
        if (!(value >= 1 && value <= 4e9))
            return MERTENS_EINVAL;
        g.ss.bucket_min = (uint32_t)value;
    } else if (!strcmp(key, "rl_fast")) {
        if (!(value == 0.0 || value == 1.0))
            return MERTENS_EINVAL;
        g.tune.rl_fast = (uint32_t)value;
    } else if (!strcmp(key, "band_lo") || !strcmp(key, "band_hi")) {
        // log2 of the band's ends; 0 (band_lo): no band
        if (!(value == 0.0 || (value >= EKW_SHIFT && value <= 31)) || value != (double)(int)value)
            return MERTENS_EINVAL;
        (key[5] == 'l' ? g.tune.band_lo : g.tune.band_hi) = (uint32_t)value;
    } else if (!strcmp(key, "update_window")) {
        if (!(value == 0.0 || (value >= 17 && value <= 40)) || value != (double)(int)value)
            return MERTENS_EINVAL;
        g.tune.update_window = (uint32_t)value;
    } else if (!strcmp(key, "sieve_ahead")) {
        if (!(value >= 1 && value <= 256))
            return MERTENS_EINVAL;
        g.tune.sieve_ahead = (uint32_t)value;
    } else if (!strcmp(key, "waves_per_cu")) {
        if (!(value >= 4 && value <= 64))
            return MERTENS_EINVAL;
        g.tune.waves_per_cu = (uint32_t)value;
    } else if (!strcmp(key, "block_auto")) {
        if (!(value >= SEG && value <= 2147483648.0) || value != std::floor(value) ||
            ((uint64_t)value) % SEG != 0)
            return MERTENS_EINVAL;
        g.tune.block_auto = (uint64_t)value;
    } else if (!strcmp(key, "serve_capacity")) {
        if (!(value >= 1 && value <= (1 << 20)))
            return MERTENS_EINVAL;
        std::lock_guard<std::mutex> lk(g.srv.mu);
        g.serve_capacity = (size_t)value;
    } else if (!strcmp(key, "serve_short_blocks")) {
        if (!(value >= 0 && value <= 1e9))
            return MERTENS_EINVAL;
        std::lock_guard<std::mutex> lk(g.srv.mu);
        g.serve_short_blocks = (uint64_t)value;
    } else if (!strcmp(key, "serve_x_budget")) {
        if (!(value >= 1 && value <= 1e12))
            return MERTENS_EINVAL;
        std::lock_guard<std::mutex> lk(g.srv.mu);
        g.serve_x_budget = (uint64_t)value;
    } else {
        return MERTENS_EINVAL;
    }
    return 0;
}

int mertens_get_param(const char *key, double *value)
{
    if (!key || !value)
        return MERTENS_EINVAL;
    const Tuning &t = g.tune;
    if (!strcmp(key, "u_scale"))
        *value = t.u_scale;
    else if (!strcmp(key, "graph"))
        *value = t.graph ? 1.0 : 0.0;
    else if (!strcmp(key, "progress"))
        *value = (double)t.progress;
    else if (!strcmp(key, "wide_bits"))
        *value = t.wide_bits;
    else if (!strcmp(key, "beta"))
        *value = t.beta;
    else if (!strcmp(key, "ychunk"))
        *value = t.ychunk;
    else if (!strcmp(key, "kchunk"))
        *value = t.kchunk;
    else if (!strcmp(key, "kbal"))
        *value = t.kbal;
    else if (!strcmp(key, "bucket_min"))
        *value = g.ss.bucket_min;
    else if (!strcmp(key, "rl_fast"))
        *value = t.rl_fast;
    else if (!strcmp(key, "update_window"))
        *value = t.update_window;
    else if (!strcmp(key, "band_lo"))
        *value = t.band_lo;
    else if (!strcmp(key, "band_hi"))
        *value = t.band_hi;
    else if (!strcmp(key, "sieve_ahead"))
        *value = t.sieve_ahead;
    else if (!strcmp(key, "waves_per_cu"))
        *value = t.waves_per_cu;
    else if (!strcmp(key, "block_auto"))
        *value = (double)t.block_auto;
    else if (!strcmp(key, "tuned"))
        *value = g.tuned ? 1.0 : 0.0;
    else if (!strcmp(key, "serve_capacity"))
        *value = (double)g.serve_capacity;
    else if (!strcmp(key, "serve_short_blocks"))
        *value = (double)g.serve_short_blocks;
    else if (!strcmp(key, "serve_x_budget"))
        *value = (double)g.serve_x_budget;
    else
        return MERTENS_EINVAL;
    return 0;
}

int mertens_stats(double *vals, int cap)
{
    if (!vals || cap <= 0)
        return 0;
    const int k = std::min(cap, 22);
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

const char *mertens_last_error(void)
{
    static thread_local std::string copy;
    std::lock_guard<std::mutex> lk(g_err_mu);
    copy = g_last_error;
    return copy.c_str();
}

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

int mertens_debug_wide(const uint64_t *m_lo, const uint64_t *m_hi, const uint64_t *d,
                       size_t count, uint64_t *q_lo, uint64_t *q_hi, int op, int on_device)
{
    if (count == 0)
        return 0;
    if (!m_lo || !m_hi || !d || !q_lo || !q_hi || op < 0 || op > 2)
        return MERTENS_EINVAL;
    for (size_t i = 0; i < count; ++i) {
        if (d[i] == 0)
            return MERTENS_EINVAL;
        const unsigned __int128 m = ((unsigned __int128)m_hi[i] << 64) | m_lo[i];
        if (op == 1 && (d[i] >> 32 || m_hi[i] >> 32))
            return MERTENS_EINVAL;
        if (op == 2 && (m / d[i]) >> 50)
            return MERTENS_EINVAL;
    }
    if (!on_device) {
        for (size_t i = 0; i < count; ++i)
            host_wide(op, m_lo[i], m_hi[i], d[i], &q_lo[i], &q_hi[i]);
        return 0;
    }
    if (!g.ready)
        return MERTENS_ENODEV;
    DevBuf dml, dmh, dd, dq;
    int rc = ensure(dml, count * 8);
    if (!rc)
        rc = ensure(dmh, count * 8);
    if (!rc)
        rc = ensure(dd, count * 8);
    if (!rc)
        rc = ensure(dq, count * 16);
    std::vector<uint64_t> h;
    if (!rc) {
        hipError_t e = hipMemcpy(dml.p, m_lo, count * 8, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(dmh.p, m_hi, count * 8, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(dd.p, d, count * 8, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_debug_wide(dml.as<uint64_t>(), dmh.as<uint64_t>(), dd.as<uint64_t>(),
                                  dq.as<uint64_t>(), count, op, g.stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(g.stream);
        if (e == hipSuccess) {
            h.resize(2 * count);
            e = hipMemcpy(h.data(), dq.p, count * 16, hipMemcpyDeviceToHost);
        }
        if (e != hipSuccess) {
            set_error("debug_wide", e, __FILE__, __LINE__);
            rc = MERTENS_EIO;
        }
    }
    dml.release();
    dmh.release();
    dd.release();
    dq.release();
    if (rc)
        return rc;
    for (size_t i = 0; i < count; ++i) {
        q_lo[i] = h[2 * i];
        q_hi[i] = h[2 * i + 1];
    }
    return 0;
}

int mertens_debug_runsum(uint64_t n_lo, uint64_t n_hi, uint64_t L, uint64_t *s_out)
{
    if (!s_out || L == 0 || (n_hi >> 18))
        return MERTENS_EINVAL;
    const unsigned __int128 N = ((unsigned __int128)n_hi << 64) | n_lo;
    const unsigned __int128 ym = N / (L + 1);
    if (ym == 0 || (ym >> 50)) {
        set_error_text("runsum needs 1 <= n/(L+1) < 2^50");
        return MERTENS_EINVAL;
    }
    if (!g.ready)
        return MERTENS_ENODEV;
    const uint64_t ymax = (uint64_t)ym;
    hipStream_t s = g.stream;
    RCCHK(g.ss.ensure_primes(std::max<uint64_t>(ceil_sqrt_host(ymax), 1024)));
    RCCHK(g.ss.ensure_pattern());
    const uint64_t B = choose_block(g.block_req, ymax);
    RCCHK(g.ss.ensure_blocks(B, 1));
    RCCHK(ensure(g.iv_small, 64));
    uint64_t *acc = g.iv_small.as<uint64_t>() + 7;
    RCCHK(g.ss.reset_carry(s));
    HIPCHK(launch_zero_u64(acc, 1, s));
    const uint64_t nblocks = ymax / B + 1;
    for (uint64_t bi = 0; bi < nblocks; ++bi) {
        const uint64_t y1 = bi * B, y2 = std::min(y1 + B - 1, ymax);
        const BlockArgs blk = g.ss.make_block(y1, y2);
        RCCHK(g.ss.sieve(blk, s, nullptr));
        HIPCHK(launch_debug_runsum(blk, n_lo, n_hi, ymax, L, acc, s));
        if (g.tune.progress && (bi + 1) % g.tune.progress == 0) {
            HIPCHK(hipStreamSynchronize(s));
            fprintf(stderr, "mertens: runsum block %llu of %llu\n", (unsigned long long)(bi + 1),
                    (unsigned long long)nblocks);
            fflush(stderr);
        }
    }
    HIPCHK(hipMemcpyAsync(s_out, acc, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return 0;
}

int mertens_debug_primes(uint64_t limit, uint64_t *count, uint64_t *last, uint64_t *sum)
{
    if (!count || !last || !sum || limit > (1ull << 32))
        return MERTENS_EINVAL;
    std::vector<uint32_t> pr;
    host_primes(limit, pr);
    *count = pr.size();
    *last = pr.empty() ? 0 : pr.back();
    uint64_t t = 0;
    for (uint32_t p : pr)
        t += p;
    *sum = t;
    return 0;
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
    RCCHK(g.ss.ensure_primes(std::max<uint64_t>(ceil_sqrt_host(yend), 1024)));
    const uint64_t B = 1ull << 30;
    RCCHK(g.ss.ensure_blocks(B));
    DevBuf dmu, dm;
    int rc = ensure(dmu, count);
    if (!rc)
        rc = ensure(dm, count * 8);
    if (rc) {
        dmu.release();
        dm.release();
        return rc;
    }
    hipError_t e = hipSuccess;
    if (g.ss.reset_carry(g.stream) != 0)
        e = hipErrorUnknown;
    for (uint64_t y = start; e == hipSuccess && y <= yend; y += B) {
        const uint64_t y2 = std::min(y + B - 1, yend);
        const BlockArgs b = g.ss.make_block(y, y2);
        if (g.ss.sieve(b, g.stream, nullptr) != 0) {
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
