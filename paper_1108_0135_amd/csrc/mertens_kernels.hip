// HIP kernels (gfx950) of the exact Mertens method of arXiv:1108.0135.
//
// Section 2 of the paper: with A[x] = M(floor(n/x)) for x <= L = floor(n/u),
// each A[x] = 1 - S[x] - sum_{k=2}^{floor(L/x)} A[kx], where S[x] collects
// every term M(floor(m/k)), m = floor(n/x), whose argument is below u and
// therefore comes from the sieve.  Section 3: y is swept in blocks; each
// block is sieved (Moebius log-prime sieve), summed into M(y), and its
// contributions are pushed into the S array; a final pass computes A.
//
// Per x the S sum is split at K = max(k0-1, floor(beta*sqrt(m)), floor(m/2^32))
// with k0 = floor(L/x)+1 and Y = floor(m/(K+1)):
//   explicit k part:   sum_{k=k0}^{K} M(floor(m/k))                  (gathers)
//   run-length part:   sum_{y=1}^{Y-1} (floor(m/y)-floor(m/(y+1))) M(y)
//                      + (floor(m/Y) - K) M(Y)
// The run-length part is evaluated in its summed-by-parts form
//   sum_{y=1}^{Y} floor(m/y) mu(y)  -  K M(Y),
// the same integer (Abel summation of the run-length weights), which needs
// mu(y) instead of M(y) and no multiply per pair.  All sums wrap mod 2^64.
#include "mertens_internal.h"

namespace mrt {

// ====================================================================
// Division by run-time invariant integers (Granlund & Montgomery, PLDI
// 1994, Fig. 4.1, N = 64): for 1 <= d < 2^32,
//   l = ceil(log2 d), mul = floor(2^64 (2^l - d) / d) + 1,
//   floor(n/d) = (t + ((n - t) >> sh1)) >> sh2,  t = mulhi(mul, n),
//   sh1 = min(l, 1), sh2 = max(l - 1, 0).
// The paper (Section 3) replaces per-pair 64-bit division by such
// multiply/shift sequences with per-divisor constants.
// ====================================================================

// floor(num / d) for num < d * 2^32 (quotient below 2^32), exact: an fp64
// estimate within 2^-19 of the true quotient, then one correction step.
__host__ __device__ inline uint64_t div_small_quot(uint64_t num, uint32_t d, uint64_t *rem)
{
    const double qd = (double)num / (double)d;
    uint64_t q = (uint64_t)qd;
    int64_t r = (int64_t)(num - q * (uint64_t)d);
    if (r < 0) {
        q -= 1;
        r += d;
    } else if (r >= (int64_t)d) {
        q += 1;
        r -= d;
    }
    *rem = (uint64_t)r;
    return q;
}

__host__ __device__ inline void gm_magic(uint32_t d, uint64_t &mul, uint32_t &sh1, uint32_t &sh2)
{
    if (d <= 1) {  // d = 1 (d = 0 never divides; mapped to 1 harmlessly)
        mul = 1;
        sh1 = 0;
        sh2 = 0;
        return;
    }
#ifdef __HIP_DEVICE_COMPILE__
    const uint32_t l = 32u - (uint32_t)__clz((int)(d - 1u));
#else
    const uint32_t l = 32u - (uint32_t)__builtin_clz(d - 1u);
#endif
    const uint64_t r = (l == 32 ? (1ull << 32) : (1ull << l)) - d;  // 2^l - d < d
    uint64_t rem;
    const uint64_t q1 = div_small_quot(r << 32, d, &rem);
    const uint64_t q2 = div_small_quot(rem << 32, d, &rem);
    mul = (q1 << 32) + q2 + 1;
    sh1 = 1;
    sh2 = l - 1;
}

__host__ __device__ inline uint64_t mulhi64(uint64_t a, uint64_t b)
{
#ifdef __HIP_DEVICE_COMPILE__
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

__host__ __device__ inline uint64_t gm_div(uint64_t n, uint64_t mul, uint32_t sh1, uint32_t sh2)
{
    const uint64_t t = mulhi64(mul, n);
    return (t + ((n - t) >> sh1)) >> sh2;
}

void host_magic(uint32_t d, uint64_t *mul, uint32_t *sh1, uint32_t *sh2)
{
    gm_magic(d, *mul, *sh1, *sh2);
}

uint64_t host_div(uint64_t n, uint64_t mul, uint32_t sh1, uint32_t sh2)
{
    return gm_div(n, mul, sh1, sh2);
}

// ====================================================================
// small device helpers
// ====================================================================
__device__ inline uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ inline uint64_t uniform_u64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t readlane_u64(uint64_t v, uint32_t lane)
{
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t wave_min_u64(uint64_t v)
{
    for (int o = 32; o >= 1; o >>= 1) {
        const uint64_t t = __shfl_xor(v, o, 64);
        v = t < v ? t : v;
    }
    return v;
}

__device__ inline uint64_t wave_max_u64(uint64_t v)
{
    for (int o = 32; o >= 1; o >>= 1) {
        const uint64_t t = __shfl_xor(v, o, 64);
        v = t > v ? t : v;
    }
    return v;
}

__device__ inline uint64_t wave_sum_u64(uint64_t v)
{
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// floor(sqrt(v)) for any uint64
__device__ inline uint64_t isqrt64(uint64_t v)
{
    uint64_t r = (uint64_t)sqrt((double)v);
    while (r > 0xFFFFFFFFull || r * r > v)
        r--;
    while (r < 0xFFFFFFFFull && (r + 1) * (r + 1) <= v)
        r++;
    return r;
}

// Exclusive scan of one int64 per thread across a workgroup of NT threads.
template <int NT>
__device__ inline int64_t wg_exclusive_scan(int64_t v, int64_t *wsum, int64_t &total)
{
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    int64_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o)
            x += t;
    }
    if (lane == 63)
        wsum[wave] = x;
    __syncthreads();
    int64_t pre = 0, tot = 0;
    for (int k = 0; k < NT / 64; ++k) {
        const int64_t s = wsum[k];
        pre += (k < (int)wave) ? s : 0;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return pre + x - v;
}

// Records: per 32 consecutive y one 16-byte record {masks, M} with masks =
// (mu = +1 bits) | (mu = -1 bits) << 32 and M = M(y) just before the
// record's first y; record r sits at words[2r], words[2r + 1].  One
// 16-byte load serves any M(y).
__device__ inline int64_t M_at(const uint64_t *__restrict__ words, uint64_t off)
{
    const uint64_t r = off >> 5;
    const uint32_t bt = (uint32_t)(off & 31);
    const uint32_t lm = (2u << bt) - 1u;  // bits 0..bt (bt = 31 wraps to all ones)
    const ulonglong2 rec = *reinterpret_cast<const ulonglong2 *>(words + 2 * r);
    return (int64_t)rec.y + (int64_t)__popc((uint32_t)rec.x & lm) -
           (int64_t)__popc((uint32_t)(rec.x >> 32) & lm);
}

// Squarefree and mu = -1 masks of the 64 y of word w (records 2w, 2w + 1).
__device__ inline void word_masks(const uint64_t *__restrict__ words, uint64_t w, uint64_t &nz,
                                  uint64_t &ng)
{
    const uint64_t a = words[4 * w], c = words[4 * w + 2];
    const uint64_t pos = (a & 0xFFFFFFFFull) | (c << 32);
    ng = (a >> 32) | (c & 0xFFFFFFFF00000000ull);
    nz = pos | ng;
}

// The block's per-block values, taken from device memory.
__device__ inline BlockArgs load_block(BlockArgs b)
{
    const BlockParams p = *b.bp;
    b.y1 = p.y1;
    b.y2 = p.y2;
    b.nseg = p.nseg;
    b.n_sq = p.n_sq;
    b.n_sq_lds = p.n_sq_lds;
    b.n_sq_lane = p.n_sq_lane;
    b.pat_off = p.pat_off;
    b.n_sieve = p.n_sieve;
    b.n_bucket = p.n_bucket;
    b.n_lane = p.n_lane;
    return b;
}

// ====================================================================
// generic small kernels
// ====================================================================
__global__ void k_block_set(BlockParams p, BlockParams *cur)
{
    if (threadIdx.x == 0)
        *cur = p;
}

hipError_t launch_block_set(const BlockParams &p, BlockParams *cur, hipStream_t s)
{
    hipLaunchKernelGGL(k_block_set, dim3(1), dim3(64), 0, s, p, cur);
    return hipGetLastError();
}

__global__ void k_block_next(const BlockParams *table, BlockParams *cur, uint32_t *index)
{
    if (threadIdx.x == 0) {
        const uint32_t i = *index;
        *cur = table[i];
        *index = i + 1;
    }
}

hipError_t launch_block_next(const BlockParams *table, BlockParams *cur, uint32_t *index,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_block_next, dim3(1), dim3(64), 0, s, table, cur, index);
    return hipGetLastError();
}

__global__ void k_zero_u64(uint64_t *p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0;
}

hipError_t launch_zero_u64(uint64_t *p, size_t n, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    const size_t grid = (n + 255) / 256;
    hipLaunchKernelGGL(k_zero_u64, dim3((uint32_t)grid), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

// ====================================================================
// a0: per-x plan.  One wave per tile, lane = x.
// ====================================================================
__global__ __launch_bounds__(UPD_THREADS) void k_plan(QueryArgs q)
{
    const uint32_t tile =
        __builtin_amdgcn_readfirstlane(blockIdx.x * (UPD_THREADS / 64) + (threadIdx.x >> 6));
    const uint32_t lane = lane_id();
    if (tile >= q.ntiles)
        return;
    const uint32_t qi = q.tile_q[tile];
    const uint32_t nx = q.tile_nx[tile];
    const uint32_t x0 = q.tile_x0[tile];
    const bool valid = lane < nx;
    uint64_t Y = 0, ysum = 0, ksum = 0;
    if (valid) {
        const uint64_t g = q.tile_g0[tile] + lane;
        const uint64_t L = q.q_L[qi];
        // keyed entries carry x and m; plain tiles are x0, x0+1, ... of query qi
        const uint64_t x = x0 ? (uint64_t)x0 + lane : (uint64_t)q.key_x[g];
        uint64_t m;
        if (!x0) {
            m = q.x_m[g];
        } else if (x <= q.q_xb[qi]) {
            m = 0;  // a wide entry carries this x; m = 0 gives K = k0 - 1, Y = 0: no work
        } else if (q.q_nhi[qi]) {
            // floor(n / x) < 2^64 for n = nhi 2^64 + n_lo (nhi < x < 2^32), in two
            // 32-bit digit steps
            const uint64_t nlo = q.q_n[qi];
            const uint64_t a1 = (q.q_nhi[qi] << 32) | (nlo >> 32);
            const uint64_t a0 = ((a1 % x) << 32) | (nlo & 0xFFFFFFFFull);
            m = ((a1 / x) << 32) | (a0 / x);
        } else {
            m = q.q_n[qi] / x;
        }
        const uint64_t k0 = L / x + 1;
        uint64_t K = (uint64_t)(q.beta * (double)isqrt64(m));
        if (K < k0 - 1)
            K = k0 - 1;
        if (K < (m >> 32))
            K = m >> 32;
        Y = m / (K + 1);
        q.x_m[g] = m;
        q.x_K[g] = K;
        q.x_k0[g] = k0;
        q.x_Y[g] = Y;
        q.S[g] = 0;
        ysum = Y;
        ksum = K >= k0 ? K - k0 + 1 : 0;
    }
    const uint64_t ymax = wave_max_u64(Y);
    ysum = wave_sum_u64(ysum);
    ksum = wave_sum_u64(ksum);
    if (lane == 0) {
        q.tile_ymax[tile] = ymax;
        atomicAdd((unsigned long long *)&q.pair_stats[0], (unsigned long long)ysum);
        atomicAdd((unsigned long long *)&q.pair_stats[1], (unsigned long long)ksum);
    }
}

hipError_t launch_plan(const QueryArgs &q, hipStream_t s)
{
    const uint32_t grid = (q.ntiles + 3) / 4;
    hipLaunchKernelGGL(k_plan, dim3(grid), dim3(UPD_THREADS), 0, s, q);
    return hipGetLastError();
}

// ====================================================================
// a1: segmented Moebius block sieve (Section 3, modified algorithm).
// ====================================================================
// ceil(log2 p) | 1 for p >= 2
__device__ inline uint32_t log_prime(uint32_t p)
{
    return (32u - (uint32_t)__clz((int)(p - 1u))) | 1u;
}

// Per block: residues of y1 modulo every sieving prime and square; cleared
// look-back states and segment ticket for the sieve.
__global__ void k_block_setup(BlockArgs b_in)
{
    const BlockArgs b = load_block(b_in);
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0)
        *b.seg_ticket = 0;
    if (i < b.nseg) {
        b.seg_state[i] = 0;
        b.sq_cnt[i] = 0;
    }
    if (i >= b.n_sieve)
        return;
    const uint64_t p = b.pres[i].x;
    b.pres[i].y = (uint32_t)(b.y1 % p);
    if (i < b.n_sq)
        b.res2[i] = b.y1 % (p * p);
}

hipError_t launch_block_setup(const BlockArgs &b, hipStream_t s)
{
    const uint32_t n = (b.n_sieve > b.nseg ? b.n_sieve : b.nseg) + 1;
    hipLaunchKernelGGL(k_block_setup, dim3((n + 255) / 256), dim3(256), 0, s, b);
    return hipGetLastError();
}

// Large squares (SQ_LDS_P < p, p^2 <= y2; p^2 > 2^20 > SEG, so at most one
// multiple per segment), each multiple listed in its segment's bucket.  Up
// to n_sq_lane one wave per prime, lane j taking multiples j, j + 64, ... of
// p^2 in the block; from n_sq_lane on (at most 64 multiples) one lane each.
__device__ inline void square_hit(const BlockArgs &b, uint64_t o)
{
    const uint32_t sg = (uint32_t)(o / SEG);
    const uint32_t k = atomicAdd(&b.sq_cnt[sg], 1u);
    if (k < SQ_BUCKET)
        b.sq_buf[(uint64_t)sg * SQ_BUCKET + k] = (uint32_t)(o % SEG);
}

__global__ void k_square_buckets(BlockArgs b_in)
{
    const BlockArgs b = load_block(b_in);
    const uint32_t i = b.n_sq_lds + __builtin_amdgcn_readfirstlane(
                                        blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6));
    if (i >= b.n_sq_lane)
        return;
    const uint64_t p = b.pres[i].x;
    const uint64_t d = p * p;
    const uint64_t r2 = b.res2[i];
    const uint64_t span = b.y2 - b.y1;
    for (uint64_t o = (r2 ? d - r2 : 0) + lane_id() * d; o <= span; o += 64 * d)
        square_hit(b, o);
}

__global__ void k_square_buckets_lane(BlockArgs b_in)
{
    const BlockArgs b = load_block(b_in);
    const uint64_t i = b.n_sq_lane + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b.n_sq)
        return;
    const uint64_t p = b.pres[i].x;
    const uint64_t d = p * p;
    const uint64_t r2 = b.res2[i];
    const uint64_t span = b.y2 - b.y1;
    for (uint64_t o = r2 ? d - r2 : 0; o <= span; o += d)
        square_hit(b, o);
}

hipError_t launch_square_buckets(const BlockArgs &b, hipStream_t s)
{
    if (b.n_sq_lane > b.n_sq_lds) {
        const uint32_t n = b.n_sq_lane - b.n_sq_lds;  // waves
        hipLaunchKernelGGL(k_square_buckets, dim3((n + 3) / 4), dim3(256), 0, s, b);
    }
    if (b.n_sq > b.n_sq_lane) {
        const uint32_t n = b.n_sq - b.n_sq_lane;  // lanes
        hipLaunchKernelGGL(k_square_buckets_lane, dim3((n + 255) / 256), dim3(256), 0, s, b);
    }
    return hipGetLastError();
}

// Bucketed primes p > SEG (index in [n_bucket, n_sieve)): up to n_lane, wave
// v of workgroup w takes the primes n_bucket + w * 16 + v + j * BK_WGS * 16,
// its lanes the multiples lane, lane + 64, ... (at most B / p <= 2^14 of
// them); the primes from n_lane on (p > span / 64) take one lane each.
// Pass 1 counts the workgroup's hits per segment in LDS and stores the
// counts; k_bucket_columns / k_bucket_starts turn them into each
// workgroup's first entry per segment; pass 2 writes the entries there.
__device__ inline uint32_t bucket_entry(uint64_t o, uint32_t lp)
{
    return (uint32_t)(o % SEG) | (lp << 17);
}

// Fill-pass entry in a group: offset in the group (24 bits) | log << 24.
__device__ inline uint32_t group_entry(uint64_t o, uint32_t lp)
{
    return (uint32_t)(o & ((1u << BK_GROUP_SHIFT) - 1)) | (lp << BK_GROUP_SHIFT);
}

// The first staged entry of workgroup w in group g is the group's first
// entry, bk_start[g * BK_GROUP_SEGS], plus the counts of workgroups before w
// over the group's segments (bk_cnt holds those per segment once
// k_bucket_columns has run); both kernels below add them up with LDS atomics.

// Count pass (FILL = false): the workgroup's hits per segment, into bk_cnt.
// Fill pass: every hit into the workgroup's run of its 2^24-y group in
// bk_stage, in the group-major layout k_bucket_regroup reads (so each
// workgroup appends to at most MAX_GROUPS runs at a time, which the L2
// gathers into whole lines).
template <bool FILL>
__global__ __launch_bounds__(BK_THREADS) void k_prime_buckets(BlockArgs b_in)
{
    const BlockArgs b = load_block(b_in);
    __shared__ uint32_t cnt[MAX_SEGS];
    if (b.n_bucket >= b.n_sieve)
        return;
    const uint32_t tid = threadIdx.x, w = blockIdx.x;
    uint32_t *mine = b.bk_cnt + (size_t)w * b.nseg;
    if (FILL) {
        const uint32_t ng = (b.nseg + BK_GROUP_SEGS - 1) / BK_GROUP_SEGS;
        for (uint32_t g = tid; g < ng; g += BK_THREADS)
            cnt[g] = b.bk_start[g * BK_GROUP_SEGS];
        __syncthreads();
        for (uint32_t sg = tid; sg < b.nseg; sg += BK_THREADS)
            atomicAdd(&cnt[sg / BK_GROUP_SEGS], mine[sg]);
    } else {
        for (uint32_t sg = tid; sg < b.nseg; sg += BK_THREADS)
            cnt[sg] = 0u;
    }
    __syncthreads();
    const uint64_t span = (uint64_t)b.nseg * SEG;
    constexpr uint32_t WAVES = BK_THREADS / 64;
    const uint32_t lane = lane_id();
    const uint32_t v = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (uint64_t i = b.n_bucket + (uint64_t)w * WAVES + v; i < b.n_lane;
         i += (uint64_t)BK_WGS * WAVES) {
        const uint2 e = b.pres[i];
        const uint64_t p = e.x;
        const uint32_t lp = log_prime(e.x);
        for (uint64_t o = (e.y ? p - e.y : 0) + lane * p; o < span; o += 64 * p) {
            if (FILL) {
                const uint32_t k = atomicAdd(&cnt[o >> BK_GROUP_SHIFT], 1u);
                b.bk_stage[k] = group_entry(o, lp);
            } else {
                atomicAdd(&cnt[o / SEG], 1u);
            }
        }
    }
    // primes above span / 64 (at most 64 multiples in the block): one lane each
    for (uint64_t i = b.n_lane + (uint64_t)w * BK_THREADS + tid; i < b.n_sieve;
         i += (uint64_t)BK_WGS * BK_THREADS) {
        const uint2 e = b.pres[i];
        const uint64_t p = e.x;
        const uint32_t lp = log_prime(e.x);
        for (uint64_t o = e.y ? p - e.y : 0; o < span; o += p) {
            if (FILL) {
                const uint32_t k = atomicAdd(&cnt[o >> BK_GROUP_SHIFT], 1u);
                b.bk_stage[k] = group_entry(o, lp);
            } else {
                atomicAdd(&cnt[o / SEG], 1u);
            }
        }
    }
    if (!FILL) {
        __syncthreads();
        for (uint32_t sg = tid; sg < b.nseg; sg += BK_THREADS)
            mine[sg] = cnt[sg];
    }
}

// Second level: workgroup (w, g) moves fill-pass workgroup w's run of group
// g from bk_stage to the per-segment lists of bk_buf (segment sg's entries
// of w start at bk_start[sg] + bk_cnt[w][sg]).  It takes the run in chunks
// of RG_CHUNK entries, sorts each chunk by segment in LDS (count with ranks,
// scan, scatter) and writes it out in that order, so consecutive threads
// write consecutive words of one segment's list.
constexpr uint32_t RG_THREADS = 512, RG_CHUNK = 8192, RG_PER = RG_CHUNK / RG_THREADS;

__global__ __launch_bounds__(RG_THREADS) void k_bucket_regroup(BlockArgs b_in)
{
    const BlockArgs b = load_block(b_in);
    __shared__ uint32_t pos[BK_GROUP_SEGS];  // next bk_buf index per segment
    __shared__ uint32_t cnt[BK_GROUP_SEGS];  // entries per segment in the chunk
    __shared__ uint32_t off[BK_GROUP_SEGS];  // their first index in `sorted`
    __shared__ uint32_t range[2];
    __shared__ uint32_t sorted[RG_CHUNK];
    if (b.n_bucket >= b.n_sieve)
        return;
    const uint32_t ng = (b.nseg + BK_GROUP_SEGS - 1) / BK_GROUP_SEGS;
    const uint32_t w = blockIdx.x % BK_WGS, g = blockIdx.x / BK_WGS;
    if (g >= ng)
        return;
    const uint32_t tid = threadIdx.x, s0 = g * BK_GROUP_SEGS;
    const uint32_t s1 = s0 + BK_GROUP_SEGS < b.nseg ? s0 + BK_GROUP_SEGS : b.nseg;
    const bool last = w + 1 == BK_WGS;
    constexpr uint32_t OMASK = (1u << BK_GROUP_SHIFT) - 1;
    if (tid == 0) {
        range[0] = b.bk_start[s0];
        range[1] = last ? b.bk_start[s1] : b.bk_start[s0];
    }
    if (tid < BK_GROUP_SEGS)
        pos[tid] = 0;
    __syncthreads();
    if (tid < BK_GROUP_SEGS && s0 + tid < s1) {
        const uint32_t *pre = b.bk_cnt + (size_t)w * b.nseg + s0 + tid;
        pos[tid] = b.bk_start[s0 + tid] + pre[0];
        atomicAdd(&range[0], pre[0]);
        if (!last)
            atomicAdd(&range[1], pre[b.nseg]);
    }
    __syncthreads();
    const uint32_t r0 = range[0], r1 = range[1];
    for (uint32_t c0 = r0; c0 < r1; c0 += RG_CHUNK) {
        const uint32_t n = r1 - c0 < RG_CHUNK ? r1 - c0 : RG_CHUNK;
        if (tid < BK_GROUP_SEGS)
            cnt[tid] = 0;
        __syncthreads();
        uint32_t val[RG_PER], rank[RG_PER];
#pragma unroll
        for (uint32_t k = 0; k < RG_PER; ++k) {
            const uint32_t i = k * RG_THREADS + tid;
            val[k] = i < n ? b.bk_stage[c0 + i] : 0u;
            rank[k] = i < n ? atomicAdd(&cnt[(val[k] & OMASK) / SEG], 1u) : 0u;
        }
        __syncthreads();
        if (tid < 64) {  // exclusive scan of the 128 counts, two per lane
            const uint32_t a = cnt[2 * tid], c = cnt[2 * tid + 1];
            uint32_t x = a + c;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = __shfl_up(x, o, 64);
                if (tid >= (uint32_t)o)
                    x += t;
            }
            off[2 * tid] = x - a - c;
            off[2 * tid + 1] = x - c;
        }
        __syncthreads();
#pragma unroll
        for (uint32_t k = 0; k < RG_PER; ++k) {
            const uint32_t i = k * RG_THREADS + tid;
            if (i < n)
                sorted[off[(val[k] & OMASK) / SEG] + rank[k]] = val[k];
        }
        __syncthreads();
        for (uint32_t i = tid; i < n; i += RG_THREADS) {
            const uint32_t v = sorted[i];
            const uint32_t o = v & OMASK, sg = o / SEG;
            b.bk_buf[pos[sg] + (i - off[sg])] = (o % SEG) | ((v >> BK_GROUP_SHIFT) << 17);
        }
        __syncthreads();
        if (tid < BK_GROUP_SEGS)
            pos[tid] += cnt[tid];
        __syncthreads();
    }
}

// Per segment (one thread each): exclusive prefix of the workgroups' counts
// (in place) and the segment's total, into bk_start.
__global__ void k_bucket_columns(BlockArgs b_in)
{
    const BlockArgs b = load_block(b_in);
    const uint32_t sg = blockIdx.x * blockDim.x + threadIdx.x;
    if (b.n_bucket >= b.n_sieve || sg >= b.nseg)
        return;
    uint32_t tot = 0;
    for (uint32_t w = 0; w < BK_WGS; ++w) {
        uint32_t *c = b.bk_cnt + (size_t)w * b.nseg + sg;
        const uint32_t v = *c;
        *c = tot;
        tot += v;
    }
    b.bk_start[sg] = tot;
}

// Segment totals -> each segment's first entry (exclusive prefix), and the
// total at [nseg].
__global__ __launch_bounds__(SIEVE_THREADS) void k_bucket_starts(BlockArgs b_in)
{
    const BlockArgs b = load_block(b_in);
    __shared__ int64_t wsum[SIEVE_THREADS / 64];
    if (b.n_bucket >= b.n_sieve)
        return;
    const uint32_t tid = threadIdx.x;
    uint64_t base = 0;
    for (uint32_t s0 = 0; s0 < b.nseg; s0 += SIEVE_THREADS) {
        const uint32_t sg = s0 + tid;
        const uint32_t tot = sg < b.nseg ? b.bk_start[sg] : 0u;
        int64_t all;
        const int64_t ex = wg_exclusive_scan<SIEVE_THREADS>((int64_t)tot, wsum, all);
        if (sg < b.nseg)
            b.bk_start[sg] = (uint32_t)(base + (uint64_t)ex);
        base += (uint64_t)all;
    }
    if (tid == 0) {
        b.bk_start[b.nseg] = (uint32_t)base;
        atomicAdd(reinterpret_cast<unsigned long long *>(b.bk_total), base);
    }
}

hipError_t launch_prime_buckets(const BlockArgs &b, hipStream_t s, hipEvent_t fill0,
                                hipEvent_t fill1, hipEvent_t fill2)
{
    if (b.n_bucket >= b.n_sieve)
        return hipSuccess;
    hipLaunchKernelGGL(k_prime_buckets<false>, dim3(BK_WGS), dim3(BK_THREADS), 0, s, b);
    hipLaunchKernelGGL(k_bucket_columns, dim3((b.nseg + 255) / 256), dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_bucket_starts, dim3(1), dim3(SIEVE_THREADS), 0, s, b);
    hipError_t e = hipSuccess;
    if (fill0)
        e = hipEventRecord(fill0, s);
    hipLaunchKernelGGL(k_prime_buckets<true>, dim3(BK_WGS), dim3(BK_THREADS), 0, s, b);
    if (fill1 && e == hipSuccess)
        e = hipEventRecord(fill1, s);
    const uint32_t ng = (b.nseg + BK_GROUP_SEGS - 1) / BK_GROUP_SEGS;
    hipLaunchKernelGGL(k_bucket_regroup, dim3(BK_WGS * ng), dim3(RG_THREADS), 0, s, b);
    if (fill2 && e == hipSuccess)
        e = hipEventRecord(fill2, s);
    const hipError_t l = hipGetLastError();
    return l != hipSuccess ? l : e;
}

// Look-back states of the fused scan.
constexpr uint64_t SEG_AGG = 1ull << 62, SEG_INCL = 2ull << 62;
constexpr uint64_t SEG_VAL = (1ull << 62) - 1;

__device__ inline void seg_publish(uint64_t *st, uint32_t seg, uint64_t flag, int64_t v)
{
    __hip_atomic_store(st + seg, flag | ((uint64_t)v & SEG_VAL), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// M(y) just before segment seg (> 0), by wave 0 of its workgroup: the
// lanes read the states of the 64 nearest unsummed predecessors and add
// totals up to the first end-of-segment value.  Every predecessor holds an
// earlier ticket, so it is running or done and its state arrives; segment
// 0 always publishes its end value, which ends the walk.
__device__ inline int64_t seg_lookback(const uint64_t *st, uint32_t seg)
{
    const uint32_t lane = lane_id();
    int64_t acc = 0;
    int64_t j = (int64_t)seg - 1;
    for (;;) {
        const int64_t idx = j - (int64_t)lane;
        uint64_t v = 0;
        if (idx >= 0)
            v = __hip_atomic_load(st + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t flag = v >> 62;
        const uint64_t notready = __ballot(flag == 0);
        const uint64_t incl = __ballot(flag == 2);
        const uint32_t nr = notready ? (uint32_t)__builtin_ctzll(notready) : 64u;
        const uint32_t fi = incl ? (uint32_t)__builtin_ctzll(incl) : 64u;
        const uint32_t use = fi < nr ? fi + 1 : nr;
        const int64_t val = (int64_t)(v << 2) >> 2;
        acc += (int64_t)wave_sum_u64(lane < use ? (uint64_t)val : 0ull);
        if (fi < nr)
            return acc;
        j -= use;
        if (use == 0)
            __builtin_amdgcn_s_sleep(2);
    }
}

// The sieve of Section 3 with the corrected log rule.  LDS holds one byte
// per y of a segment of SEG consecutive y: bits 0-6 accumulate
// l_p = ceil(log2 p)|1 over the sieving primes p | y on top of a bias of
// 64 - floor(log2 y), bit 7 flags a square divisor.  With A the log sum and
// T = floor(log2 y), the byte holds A + 64 - T < 128 (A < T + 1 + 2 omega(y)),
// so bytes never carry into each other and:
//   bit 7 set                           -> mu = 0
//   bit 6 set (A >= T, fully split)     -> mu = (-1)^A
//   otherwise (one prime above Psieve)  -> mu = -(-1)^A
// where A's parity (every l_p is odd) is bit 0 flipped when T is odd.
//
// Layout: 32-y group G (one record) holds y offsets 32G + t in eight
// 32-bit words, offset t in word t & 7, byte t >> 3.  The bits 7, 6 and 0
// of the eight words then gather into the group's 32-bit masks in y order
// by shifts alone.  A prime walk with step 64p keeps both the byte and the
// word within its group, so it advances by a constant 64p bytes.
//
// Each workgroup sieves SV_R consecutive segments (a group of segments
// claimed in ticket order) with one residue per prime: the small primes'
// and small squares' (one wavefront per prime) first multiples in every
// segment of the group are set up at the start in lane-distributed
// registers; the first SV_U * SIEVE_THREADS larger primes (one lane per
// prime) carry their next offset in per-thread registers.  The classified masks of
// all SV_R segments stay in registers until the group's M(y) prefix is
// known (workgroup scan plus decoupled look-back over earlier groups);
// then whole 16-byte records are written.
constexpr int SV_R = 4;
constexpr int SV_U = 16;
constexpr uint32_t SV_GROUPS = SEG / 32;                  // records per segment
constexpr int SV_GPT = (int)(SV_GROUPS / SIEVE_THREADS);  // records per thread and segment
static_assert(SV_GPT == 4, "four 16-bit count fields per thread and segment");

// Byte address (in the segment's LDS) of the word holding y offset o, and
// the shift of o's byte within it.
__device__ inline uint32_t sv_addr(uint32_t o)
{
    // (o & ~31) | ((o & 7) << 2) as one bit-field insert of 4o into o (the
    // compiler would spend two masks and an add on it)
    uint32_t a;
    __asm__("v_bfi_b32 %0, 31, %1, %2" : "=v"(a) : "v"(o << 2), "v"(o));
    return a;
}
__device__ inline uint32_t sv_shift(uint32_t o)
{
    return o & 24u;
}
__device__ inline void sv_add(uint8_t *lb, uint32_t o, uint32_t v)
{
    atomicAdd(reinterpret_cast<uint32_t *>(lb + sv_addr(o)), v << sv_shift(o));
}
__device__ inline void sv_square(uint8_t *lb, uint32_t o)
{
    atomicOr(reinterpret_cast<uint32_t *>(lb + sv_addr(o)), 0x80u << sv_shift(o));
}

// The multiples o = f + p (lane + 64 i) < SEG of one prime (or square) p
// taken by a whole wave (f, p wave-uniform; f < p).  A step of 64p keeps
// each lane's byte and word within its 32-y group, so the word address
// advances by 64p; the wave runs while lane 63's multiple (the largest) is
// in the segment, a count kept in scalar registers, and then each lane
// takes at most one more (its next multiple passes lane 63's last).
template <bool SQUARE>
__device__ inline void sv_wave_walk(uint8_t *lb, uint32_t f, uint32_t p, uint32_t lp,
                                    uint32_t lane)
{
    const uint32_t o = f + __umul24(lane, p);
    const uint32_t step = 64u * p;
    const uint32_t v = (SQUARE ? 0x80u : lp) << sv_shift(o);
    uint32_t a = sv_addr(o);
    for (uint32_t o63 = f + 63u * p; o63 < SEG; o63 += step) {
        if (SQUARE)
            atomicOr(reinterpret_cast<uint32_t *>(lb + a), v);
        else
            atomicAdd(reinterpret_cast<uint32_t *>(lb + a), v);
        a += step;
    }
    if (a < SEG) {
        if (SQUARE)
            atomicOr(reinterpret_cast<uint32_t *>(lb + a), v);
        else
            atomicAdd(reinterpret_cast<uint32_t *>(lb + a), v);
    }
}

// mu masks of one 32-y group from its eight LDS words: pos (mu = +1) and
// neg (mu = -1), bit t for y offset t; tpar = ~0 when T is odd.
__device__ inline void sv_classify(const uint4 lo, const uint4 hi, uint32_t tpar, uint32_t &pos,
                                   uint32_t &neg)
{
    const uint32_t w[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    uint32_t sq = 0, fu = 0, pa = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t m = 0x01010101u << k;
        sq |= (w[k] >> (7 - k)) & m;
        fu |= (k < 7 ? (w[k] >> (6 - k)) : (w[k] << 1)) & m;
        pa |= (w[k] << k) & m;
    }
    const uint32_t nz = ~sq;
    neg = nz & ~(fu ^ pa ^ tpar);
    pos = nz & ~neg;
}

// The record of y in [0, 32): mu by trial division (y = 0 is a multiple of
// every sieving prime, so its byte overflows and carries into the bytes of
// y = 8, 16, 24 of the same word; mu(0) = 0 by convention).  Below 32 the
// part left after removing 2, 3 and 5 is 1 or a prime.
__device__ inline void sv_classify_first(uint32_t &pos, uint32_t &neg)
{
    pos = 0;
    neg = 0;
    for (uint32_t t = 1; t < 32; ++t) {
        uint32_t v = t;
        int m = 1;
        for (uint32_t d = 2; d <= 5 && m != 0; d += (d == 2 ? 1u : 2u)) {
            if (v % d == 0) {
                v /= d;
                m = (v % d == 0) ? 0 : -m;
            }
        }
        if (m != 0 && v > 1)
            m = -m;
        if (m > 0)
            pos |= 1u << t;
        else if (m < 0)
            neg |= 1u << t;
    }
}

// Inclusive prefix over the wave of four 16-bit fields packed in a uint64.
__device__ inline uint64_t wave_scan_u64(uint64_t x)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t t = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o)
            x += t;
    }
    return x;
}

__global__ __launch_bounds__(SIEVE_THREADS) void k_sieve(BlockArgs b_in)
{
    const BlockArgs b = load_block(b_in);
    constexpr uint32_t NWAVES = SIEVE_THREADS / 64;
    __shared__ uint4 lds4[SEG / 16];
    // per (segment, record slot) and wave: wave totals, then their exclusive prefix
    __shared__ int32_t stot[SV_R * SV_GPT * NWAVES];
    __shared__ int64_t bcast[2];  // ticket, M(y) before the group
    uint8_t *lb = reinterpret_cast<uint8_t *>(lds4);
    const uint32_t tid = threadIdx.x, lane = lane_id();
    if (tid == 0)
        bcast[0] = atomicAdd(b.seg_ticket, 1u);
    __syncthreads();
    const uint32_t grp = __builtin_amdgcn_readfirstlane((uint32_t)bcast[0]);
    const uint32_t ngroups = (b.nseg + SV_R - 1) / SV_R;
    if (grp >= ngroups)
        return;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t seg0 = grp * SV_R;
    const uint32_t nsegs = b.nseg - seg0 < (uint32_t)SV_R ? b.nseg - seg0 : (uint32_t)SV_R;
    const uint32_t segbase0 = seg0 * SEG;  // < 2^31

    // ---- first multiple in each of the group's segments
    // squares p^2, p <= SQ_LDS_P (index < n_sq_lds): wave w, lane j holds
    // index 15 - w + 16 j (the squares with many multiples go to the last
    // waves, the small primes with many to the first)
    uint32_t q_p2 = 0, q_first[SV_R];
    {
        const uint32_t i = (NWAVES - 1u - wave) + NWAVES * lane;
        uint32_t f = 0, st = 0;
        if (i < b.n_sq_lds) {
            const uint32_t p = b.pres[i].x;
            q_p2 = p * p;  // < 2^21
            uint32_t r = (uint32_t)b.res2[i] + segbase0 % q_p2;
            if (r >= q_p2)
                r -= q_p2;
            f = r ? q_p2 - r : 0;
            st = SEG % q_p2;
        }
#pragma unroll
        for (int j = 0; j < SV_R; ++j) {  // next segment: (f - SEG) mod p^2
            q_first[j] = f;
            f = f >= st ? f - st : f + q_p2 - st;
        }
    }
    // small primes (index in [FIRST_SIEVED, n_small)): wave w, lane j holds
    // index FIRST_SIEVED + w + 16 j
    uint32_t s_p = 0, s_pl = 0, s_first[SV_R];
    {
        const uint32_t i = FIRST_SIEVED + wave + NWAVES * lane;
        uint32_t f = 0, st = 0;
        if (i < b.n_small) {
            const uint32_t p = b.pres[i].x;
            s_p = p;
            s_pl = p | (log_prime(p) << 24);
            uint32_t r = b.pres[i].y + segbase0 % p;  // both < p < SMALL_P
            if (r >= p)
                r -= p;
            f = r ? p - r : 0;
            st = SEG % p;
        }
#pragma unroll
        for (int j = 0; j < SV_R; ++j) {
            s_first[j] = f;
            f = f >= st ? f - st : f + s_p - st;
        }
    }
    // squares below SEG are walked by whole waves (the wave's first nq_w
    // lanes hold them, in increasing order); larger ones (at most one
    // multiple per segment) by their own lane
    const uint32_t nq_w =
        (uint32_t)__builtin_popcountll(__ballot(q_p2 != 0u && q_p2 < SEG));
    const uint32_t ns_w =
        b.n_small > FIRST_SIEVED + wave ? (b.n_small - FIRST_SIEVED - wave + NWAVES - 1) / NWAVES : 0u;
    // larger primes, one lane each: the first SV_U per thread carried
    // ({p | l_p << 24} and the next offset, which may pass SEG for p > SEG;
    // absent ones keep an offset that never comes below SEG in SV_R steps).
    // The carried primes are the 2^14 primes from SMALL_P on, all < 2^18.
    const uint32_t lp0 = b.n_small > FIRST_SIEVED ? b.n_small : FIRST_SIEVED;
    const uint32_t i_end = b.n_bucket < b.n_sieve ? b.n_bucket : b.n_sieve;
    const uint32_t i_carry =
        i_end - lp0 < (uint32_t)(SV_U * SIEVE_THREADS) ? i_end : lp0 + SV_U * SIEVE_THREADS;
    uint32_t c_pl[SV_U], c_o[SV_U];
#pragma unroll
    for (int u = 0; u < SV_U; ++u) {
        const uint32_t i = lp0 + tid + (uint32_t)u * SIEVE_THREADS;
        c_pl[u] = 0;
        c_o[u] = ~0u;
        if (i < i_carry) {
            const uint2 e = b.pres[i];  // p < 2^18 here (at most 2^14 primes past SMALL_P)
            uint32_t r = e.y + segbase0 % e.x;
            if (r >= e.x)
                r -= e.x;
            c_pl[u] = e.x | (log_prime(e.x) << 24);
            c_o[u] = r ? e.x - r : 0;
        }
    }

    uint32_t mpos[SV_R][SV_GPT], mneg[SV_R][SV_GPT];
    uint64_t wex[SV_R];  // in-wave exclusive prefix of the four records' mu sums (16-bit fields)

#pragma unroll
    for (int j = 0; j < SV_R; ++j) {
        if ((uint32_t)j >= nsegs) {
#pragma unroll
            for (int h = 0; h < SV_GPT; ++h) {
                mpos[j][h] = mneg[j][h] = 0;
                if (lane == 63)
                    stot[(j * SV_GPT + h) * NWAVES + wave] = 0;
            }
            wex[j] = 0;
            continue;
        }
        const uint32_t seg = seg0 + (uint32_t)j;
        const uint32_t segbase = seg * SEG;
        const uint64_t s0 = b.y1 + segbase;
        // T = floor(log2 y) is one value on a segment from 2^17 on; below
        // (the very first segment) it is taken per record
        const bool first_seg = s0 < SEG;
        const uint32_t Ts = 63u - (uint32_t)__clzll((long long)(s0 | 1));

        // pre-sieved pattern (2,3,5,7,11,13 and squares 4, 9) plus the bias
        uint32_t po = b.pat_off + segbase % PAT;
        if (po >= PAT)
            po -= PAT;
        // copy (po / 4) mod 8 starts 4 ((po / 4) mod 8) pattern bytes later, so
        // the segment is a whole run of 32-byte groups of it
        const uint4 *src = reinterpret_cast<const uint4 *>(
            b.pat32 + (size_t)((po >> 2) & 7u) * PAT_WORDS + (size_t)(po >> 5) * 8);
        // the next load in flight while one is biased and stored (8 uint4 per thread)
        const uint32_t bias_s = (64u - Ts) * 0x01010101u;
        constexpr int PER = (int)(SEG / 16 / SIEVE_THREADS);
        uint4 cur = src[tid];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const uint32_t q = tid + (uint32_t)k * SIEVE_THREADS;
            const uint4 nxt = (k + 1 < PER) ? src[q + SIEVE_THREADS] : cur;
            uint32_t bias = bias_s;
            if (first_seg) {
                const uint32_t yg = (uint32_t)s0 + (q >> 1) * 32;
                bias = (64u - (yg ? 31u - (uint32_t)__clz((int)yg) : 4u)) * 0x01010101u;
            }
            lds4[q] = make_uint4(cur.x + bias, cur.y + bias, cur.z + bias, cur.w + bias);
            cur = nxt;
        }
        __syncthreads();

        // squares p^2 < SEG: one wave per prime, lane i takes multiples i, i+64, ...
        for (uint32_t jj = 0; jj < nq_w; ++jj)
            sv_wave_walk<true>(lb, __builtin_amdgcn_readlane(q_first[j], jj),
                               __builtin_amdgcn_readlane(q_p2, jj), 0u, lane);
        // squares SEG < p^2 <= SQ_LDS_P^2: one lane per prime
        if (q_p2 > SEG && q_first[j] < SEG)
            sv_square(lb, q_first[j]);
        // small primes: one wave per prime, lane i takes multiples i, i+64, ...
        for (uint32_t jj = 0; jj < ns_w; ++jj) {
            const uint32_t pl = __builtin_amdgcn_readlane(s_pl, jj);
            sv_wave_walk<false>(lb, __builtin_amdgcn_readlane(s_first[j], jj), pl & 0xFFFFFFu,
                                pl >> 24, lane);
        }
        // larger primes, carried: walk, then keep the offset in the next segment
#pragma unroll
        for (int u = 0; u < SV_U; ++u) {
            const uint32_t p = c_pl[u] & 0xFFFFFFu, v = c_pl[u] >> 24;
            uint32_t o = c_o[u];
            for (; o < SEG; o += p)
                sv_add(lb, o, v);
            c_o[u] = o - SEG;
        }
        // larger primes past the carried ones: offsets from the residues
        for (uint32_t i = i_carry + tid; i < i_end; i += SIEVE_THREADS) {
            const uint2 e = b.pres[i];
            const uint32_t p = e.x, lp = log_prime(p);
            uint64_t r = (uint64_t)e.y + segbase % p;
            if (r >= p)
                r -= p;
            for (uint64_t o = r ? p - r : 0; o < SEG; o += p)
                sv_add(lb, (uint32_t)o, lp);
        }
        // bucketed primes (> SEG): their hits in this segment, listed per block
        if (b.n_bucket < b.n_sieve) {
            const uint32_t e1 = b.bk_start[seg + 1];
            for (uint32_t k = b.bk_start[seg] + tid; k < e1; k += SIEVE_THREADS) {
                const uint32_t v = b.bk_buf[k];
                sv_add(lb, v & (SEG - 1), v >> 17);
            }
        }
        // squares p^2 > SQ_LDS_P^2 (> SEG): at most one multiple each in the
        // segment, listed in its bucket.  Should the bucket have overflowed,
        // every such prime is checked here instead: f = offset of the block's
        // first multiple; the segment's first is f - segbase mod p^2, with the
        // quotient estimated in fp32 (t < 2^31, error < 1) and corrected once.
        const uint32_t nsq = b.sq_cnt[seg];
        if (nsq <= SQ_BUCKET) {
            for (uint32_t k = tid; k < nsq; k += SIEVE_THREADS)
                sv_square(lb, b.sq_buf[(uint64_t)seg * SQ_BUCKET + k]);
        }
        for (uint32_t i = b.n_sq_lds + tid; nsq > SQ_BUCKET && i < b.n_sq; i += SIEVE_THREADS) {
            const uint64_t p = b.pres[i].x;
            const uint64_t d = p * p;
            const uint64_t r2 = b.res2[i];
            const uint64_t f = r2 ? d - r2 : 0;
            uint64_t o;
            if (f >= segbase) {
                o = f - segbase;
            } else {
                const uint32_t t = segbase - (uint32_t)f;
                const uint64_t qt = (uint64_t)((float)t / (float)d);
                int64_t rem = (int64_t)t - (int64_t)(qt * d);
                if (rem < 0)
                    rem += (int64_t)d;
                else if (rem >= (int64_t)d)
                    rem -= (int64_t)d;
                o = rem ? d - (uint64_t)rem : 0;
            }
            if (o < SEG)
                sv_square(lb, (uint32_t)o);
        }
        __syncthreads();

        // classify: thread t owns records t + 1024 h of the segment
        const uint32_t tpar = (Ts & 1u) ? ~0u : 0u;
        uint64_t packed = 0;
#pragma unroll
        for (int h = 0; h < SV_GPT; ++h) {
            const uint32_t G = tid + (uint32_t)h * SIEVE_THREADS;
            uint32_t pos, neg;
            if (first_seg) {
                const uint32_t yg = (uint32_t)s0 + G * 32;
                const uint32_t T = yg ? 31u - (uint32_t)__clz((int)yg) : 4u;
                if (yg == 0)
                    sv_classify_first(pos, neg);
                else
                    sv_classify(lds4[2 * G], lds4[2 * G + 1], (T & 1u) ? ~0u : 0u, pos, neg);
            } else {
                sv_classify(lds4[2 * G], lds4[2 * G + 1], tpar, pos, neg);
            }
            mpos[j][h] = pos;
            mneg[j][h] = neg;
            const int32_t c = __popc(pos) - __popc(neg);  // in [-32, 32]
            packed |= (uint64_t)(uint32_t)(c + 64) << (16 * h);
        }
        // in-wave prefix of the four records' sums (biased fields <= 64 * 96)
        const uint64_t incl = wave_scan_u64(packed);
        wex[j] = incl - packed;
        if (lane == 63) {
#pragma unroll
            for (int h = 0; h < SV_GPT; ++h)
                stot[(j * SV_GPT + h) * NWAVES + wave] =
                    (int32_t)((incl >> (16 * h)) & 0xFFFFu) - 64 * 64;
        }
        __syncthreads();  // the next segment's pattern copy overwrites the bytes
    }

    // the zero totals of absent segments (a group shorter than SV_R) were
    // written after the last barrier
    __syncthreads();
    // exclusive prefix over (segment, record slot, wave) of the wave totals
    if (wave == 0) {
        constexpr int E = SV_R * SV_GPT * (int)NWAVES;  // 256 = 4 per lane
        int32_t v[E / 64], s = 0;
#pragma unroll
        for (int e = 0; e < E / 64; ++e) {
            v[e] = stot[lane * (E / 64) + e];
            s += v[e];
        }
        int32_t x = s;
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t t = __shfl_up(x, o, 64);
            if (lane >= (uint32_t)o)
                x += t;
        }
        int32_t run = x - s;
#pragma unroll
        for (int e = 0; e < E / 64; ++e) {
            stot[lane * (E / 64) + e] = run;
            run += v[e];
        }
        const int64_t T = __shfl(x, 63, 64);  // the group's mu sum
        int64_t before;
        if (grp == 0) {
            before = *b.carry;
        } else {
            if (lane == 0)
                seg_publish(b.seg_state, grp, SEG_AGG, T);
            before = seg_lookback(b.seg_state, grp);
        }
        if (lane == 0) {
            seg_publish(b.seg_state, grp, SEG_INCL, before + T);
            bcast[1] = before;
            if (seg0 + nsegs == b.nseg)
                *b.carry = before + T;
        }
    }
    __syncthreads();
    const int64_t P = bcast[1];
#pragma unroll
    for (int j = 0; j < SV_R; ++j) {
        if ((uint32_t)j >= nsegs)
            break;
        const uint64_t rbase = (uint64_t)(seg0 + (uint32_t)j) * SV_GROUPS + tid;
#pragma unroll
        for (int h = 0; h < SV_GPT; ++h) {
            const int32_t inwave =
                (int32_t)((wex[j] >> (16 * h)) & 0xFFFFu) - 64 * (int32_t)lane;
            const int64_t m = P + stot[(j * SV_GPT + h) * NWAVES + wave] + inwave;
            ulonglong2 *r = reinterpret_cast<ulonglong2 *>(
                b.words + 2 * (rbase + (uint64_t)h * SIEVE_THREADS));
            *r = make_ulonglong2((uint64_t)mpos[j][h] | ((uint64_t)mneg[j][h] << 32), (uint64_t)m);
        }
    }
}

hipError_t launch_sieve(const BlockArgs &b, hipStream_t s)
{
    hipLaunchKernelGGL(k_sieve, dim3((b.nseg + SV_R - 1) / SV_R), dim3(SIEVE_THREADS), 0, s, b);
    return hipGetLastError();
}

constexpr int SCAN_THREADS = 1024;

// ====================================================================
// a3: per-block contribution update.
// ====================================================================
// Prep: per x, the k range whose quotients floor(m/k) land in [y1, y2]; the
// one-off term -K*M(Y) when Y is in this block; per tile, the number of
// work items of the run-length part and of the explicit k part.
// Explicit-k pairs whose quotient lies in the band [2^wa, 2^wb) of y
// (wa < wb) are summed y-major by k_ek_window, for the tiles this predicate
// selects (m below 2^48, the 8 x 8 walk, the fused quotient rule in the
// block); the persistent update skips them.  For x with m, the band's k are
// [floor(m / 2^wb) + 1, floor(m / 2^wa)].
__device__ inline bool band_tile(const QueryArgs &q, const BlockArgs &b, uint64_t mmax,
                                 uint32_t mode)
{
    return q.rl_fast && (b.y1 == 0 || b.y2 - b.y1 < b.y1) && mmax < (1ull << 48) && mode == 0;
}

// The k of a band tile left to the persistent update lie in [tmin, amax]
// (below every x's band) and [bmin, tmax] (above it), from lane l's x (m,
// its k range [klo, khi] in the block); amax = 0 when no x has k below its
// band, bmin = ~0 when none above.  When amax + 1 >= bmin there is no gap.
__device__ inline void band_gap(uint64_t m, uint64_t klo, uint64_t khi, uint32_t wa, uint32_t wb,
                                uint64_t &amax, uint64_t &bmin)
{
    const bool has = klo <= khi;
    const uint64_t hl = (m >> wb) + 1, hh = m >> wa;
    const uint64_t ae = khi < hl - 1 ? khi : hl - 1;
    const uint64_t bs = klo > hh + 1 ? klo : hh + 1;
    amax = uniform_u64(wave_max_u64(has && klo <= ae ? ae : 0ull));
    bmin = uniform_u64(wave_min_u64(has && bs <= khi ? bs : ~0ull));
}

// Work items of a mode-0 tile's explicit-k part: chunks of kchunk k over
// [tmin, aend] (aend = amax when the band leaves a gap, else tmax), then
// over [bmin, tmax] after a gap; n_a is the count of the first run.
struct KChunks {
    uint64_t aend, bmin, n_a, n_b;
};

__device__ inline KChunks k_chunks(uint64_t tmin, uint64_t tmax, uint32_t kchunk, bool gap,
                                   uint64_t amax, uint64_t bmin)
{
    KChunks c;
    const bool split = gap && amax + 1 < bmin;
    c.aend = split ? amax : tmax;
    c.bmin = bmin;
    c.n_a = c.aend >= tmin ? (c.aend - tmin) / kchunk + 1 : 0;
    c.n_b = split && bmin <= tmax ? (tmax - bmin) / kchunk + 1 : 0;
    return c;
}

__global__ __launch_bounds__(UPD_THREADS) void k_update_prep(QueryArgs q, BlockArgs b_in, uint32_t wa,
                                                            uint32_t wb)
{
    const BlockArgs b = load_block(b_in);
    const uint32_t tile =
        __builtin_amdgcn_readfirstlane(blockIdx.x * (UPD_THREADS / 64) + (threadIdx.x >> 6));
    const uint32_t lane = lane_id();
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *q.counter = 0;
    if (tile >= q.ntiles)
        return;
    const uint32_t nx = q.tile_nx[tile];
    const uint64_t g = q.tile_g0[tile] + lane;
    const uint64_t y1e = b.y1 > 0 ? b.y1 : 1;
    uint64_t klo = 1, khi = 0, m = 0;
    if (lane < nx) {
        m = q.x_m[g];
        const uint64_t K = q.x_K[g], k0 = q.x_k0[g], Y = q.x_Y[g];
        uint64_t lo = m / (b.y2 + 1) + 1;
        if (lo < k0)
            lo = k0;
        uint64_t hi = m / y1e;
        if (hi > K)
            hi = K;
        if (lo <= hi) {
            klo = lo;
            khi = hi;
        }
        if (Y >= y1e && Y <= b.y2)
            q.S[g] -= K * (uint64_t)M_at(b.words, Y - b.y1);
    }
    if (lane < nx) {
        q.x_klo[g] = klo;
        q.x_khi[g] = khi;
    }
    const bool has = klo <= khi;
    const uint64_t kpairs = wave_sum_u64(has ? khi - klo + 1 : 0ull);
    if (lane == 0 && kpairs)
        atomicAdd((unsigned long long *)&q.pair_stats[3], (unsigned long long)kpairs);
    const uint64_t tmin = wave_min_u64(has ? klo : ~0ull);
    const uint64_t tmax = wave_max_u64(has ? khi : 0ull);
    // lane-slots the 8 x 8 walk would spend: each x-group of 8 lanes walks
    // the union of its k ranges, 8 k at a time
    uint64_t glo = has ? klo : ~0ull, ghi = has ? khi : 0ull;
    for (int o = 1; o < 8; o <<= 1) {
        const uint64_t a = __shfl_xor(glo, o, 64), c = __shfl_xor(ghi, o, 64);
        glo = a < glo ? a : glo;
        ghi = c > ghi ? c : ghi;
    }
    const uint64_t slots =
        wave_sum_u64((lane & 7u) == 0 && glo <= ghi ? 8 * (ghi - glo + 1) : 0ull);
    uint64_t nk = 0;
    uint32_t mode = 0;
    if (kpairs > 0) {
        if (q.kbal == 0 || q.kbal * kpairs >= slots) {
            mode = 0;  // the 8 x 8 walk keeps at least 1/kbal of its lanes busy
            uint64_t amax = 0, bmin = ~0ull;
            const bool gap = wa < wb && band_tile(q, b, uniform_u64(wave_max_u64(m)), 0);
            if (gap) {
                band_gap(m, klo, khi, wa, wb, amax, bmin);
                // the band's pairs (k_ek_window takes them), for the statistics
                const uint64_t hl = (m >> wb) + 1, hh = m >> wa;
                const uint64_t a = klo > hl ? klo : hl, c = khi < hh ? khi : hh;
                const uint64_t bp = wave_sum_u64(klo <= khi && a <= c ? c - a + 1 : 0ull);
                if (lane == 0 && bp)
                    atomicAdd((unsigned long long *)&q.pair_stats[4], (unsigned long long)bp);
            }
            const KChunks c = k_chunks(tmin, tmax, q.kchunk, gap, amax, bmin);
            nk = c.n_a + c.n_b;
        } else {
            mode = 1;  // balanced runs of the tile's pairs
            nk = (kpairs + K_BAL_PAIRS - 1) / K_BAL_PAIRS;
        }
    }
    if (lane == 0) {
        q.tile_klo[tile] = tmin;
        q.tile_khi[tile] = tmax;
        q.tile_mode[tile] = mode;
        const uint64_t yb = q.tile_ymax[tile] < b.y2 ? q.tile_ymax[tile] : b.y2;
        const uint64_t yal = y1e & ~63ull;
        const uint64_t nmu = yb >= y1e ? (yb - yal) / q.ychunk + 1 : 0;
        q.tile_nmu[tile] = (uint32_t)nmu;
        q.tile_items[tile] = nmu + nk;
    }
}

// ====================================================================
// Wide entries: x whose m = floor(n/x) needs more than 64 bits (n up to
// 2^96), or at least 2^wide_bits.  Same split as the plain path (Section
// 2): K = max(k0 - 1, floor(beta sqrt(m)), floor(m / 2^32)), so Y =
// floor(m/(K+1)) < 2^32 and every run-length quotient is three 32-bit
// digit steps; explicit-k quotients are below the sieve bound (< 2^64).
// ====================================================================
struct U128 {
    uint64_t lo, hi;
};

__host__ __device__ inline bool u128_less(U128 a, U128 b)
{
    return a.hi != b.hi ? a.hi < b.hi : a.lo < b.lo;
}

__host__ __device__ inline U128 mul64(uint64_t a, uint64_t b)
{
    return U128{a * b, mulhi64(a, b)};
}

// floor(a / d) for any a and d >= 1, one quotient bit per step (used once per
// entry and block only).
__host__ __device__ inline U128 udiv128_bits(U128 a, uint64_t d)
{
    U128 q{0, 0};
    uint64_t r = 0;
    for (int i = 127; i >= 0; --i) {
        const uint64_t bit = i >= 64 ? (a.hi >> (i - 64)) & 1u : (a.lo >> i) & 1u;
        const bool carry = r >> 63;  // r * 2 + bit would not fit 64 bits
        r = (r << 1) | bit;
        if (carry || r >= d) {
            r -= d;  // the true value minus d is below d, so wrapping is exact
            if (i >= 64)
                q.hi |= 1ull << (i - 64);
            else
                q.lo |= 1ull << i;
        }
    }
    return q;
}

// One digit step: floor(a / y) and a mod y for a < y 2^32, y < 2^32, from an
// fp64 estimate (error below one) and one integer correction.
__host__ __device__ inline uint64_t digit_div(uint64_t a, uint64_t y, double rcp, uint64_t &r)
{
    uint64_t q = (uint64_t)((double)a * rcp);
    r = a - q * y;
    if ((int64_t)r < 0) {
        --q;
        r += y;
    } else if (r >= y) {
        ++q;
        r -= y;
    }
    return q;
}

// floor(m / y) mod 2^64 for m < 2^96 and 1 <= y < 2^32.
__host__ __device__ inline uint64_t wide_quot_low(U128 m, uint64_t y)
{
    const double rcp = 1.0 / (double)y;
    uint64_t r;
    (void)digit_div(m.hi, y, rcp, r);
    const uint64_t q1 = digit_div((r << 32) | (m.lo >> 32), y, rcp, r);
    const uint64_t q0 = digit_div((r << 32) | (m.lo & 0xFFFFFFFFull), y, rcp, r);
    return (q1 << 32) + q0;
}

// floor(m / k) for a quotient below 2^50: fp64 estimate, then the exact
// 128-bit check either way.
__host__ __device__ inline uint64_t wide_quot_small(U128 m, double md, uint64_t k)
{
    uint64_t q = (uint64_t)(md / (double)k);
    if (u128_less(m, mul64(k, q)))
        --q;
    else if (!u128_less(m, mul64(k, q + 1)))
        ++q;
    return q;
}

// The wide helpers on one argument, for the diagnostic entry point:
// op 0: floor(m/d) (128 bits, any d >= 1); op 1: floor(m/d) mod 2^64 by digit
// steps (m < 2^96, d < 2^32); op 2: floor(m/d) by fp64 estimate and exact
// check (quotient < 2^50).
__host__ __device__ inline void wide_op(int op, uint64_t mlo, uint64_t mhi, uint64_t d,
                                        uint64_t &qlo, uint64_t &qhi)
{
    const U128 m{mlo, mhi};
    qhi = 0;
    if (op == 0) {
        const U128 q = udiv128_bits(m, d);
        qlo = q.lo;
        qhi = q.hi;
    } else if (op == 1) {
        qlo = wide_quot_low(m, d);
    } else {
        qlo = wide_quot_small(m, (double)mhi * 18446744073709551616.0 + (double)mlo, d);
    }
}

void host_wide(int op, uint64_t mlo, uint64_t mhi, uint64_t d, uint64_t *qlo, uint64_t *qhi)
{
    wide_op(op, mlo, mhi, d, *qlo, *qhi);
}

__global__ void k_debug_wide(const uint64_t *mlo, const uint64_t *mhi, const uint64_t *d,
                             uint64_t *out, size_t count, int op)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        wide_op(op, mlo[i], mhi[i], d[i], out[2 * i], out[2 * i + 1]);
}

hipError_t launch_debug_wide(const uint64_t *mlo, const uint64_t *mhi, const uint64_t *d,
                             uint64_t *out, size_t count, int op, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_debug_wide, dim3((uint32_t)((count + 255) / 256)), dim3(256), 0, s, mlo,
                       mhi, d, out, count, op);
    return hipGetLastError();
}

// Diagnostic: the sum over k > L of M(floor(n/k)) for one argument n < 2^82,
// grouped by y = floor(n/k) with plain weights floor(n/y) - floor(n/(y+1))
// (floor(n/ymax) - L at y = ymax), all mod 2^64; no split, no explicit k.
// Every quotient is taken mod 2^64: by 32-bit digit steps for y < 2^32,
// else by the fp64 estimate with the exact 128-bit check (quotient < 2^50).
__device__ inline uint64_t quot_low_any(U128 n, double nd, uint64_t y)
{
    return y < (1ull << 32) ? wide_quot_low(n, y) : wide_quot_small(n, nd, y);
}

__global__ __launch_bounds__(256) void k_debug_runsum(BlockArgs b_in, uint64_t nlo, uint64_t nhi,
                                                      uint64_t ymax, uint64_t L, uint64_t *acc)
{
    const BlockArgs b = load_block(b_in);
    const U128 n{nlo, nhi};
    const double nd = (double)nhi * 18446744073709551616.0 + (double)nlo;
    const uint64_t y1e = b.y1 > 0 ? b.y1 : 1;
    const uint64_t yhi = b.y2 < ymax ? b.y2 : ymax;
    uint64_t s = 0;
    for (uint64_t y = y1e + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; y <= yhi;
         y += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t qy = quot_low_any(n, nd, y);
        const uint64_t w = y < ymax ? qy - quot_low_any(n, nd, y + 1) : qy - L;
        s += w * (uint64_t)M_at(b.words, y - b.y1);
    }
    s = wave_sum_u64(s);
    if (lane_id() == 0 && s)
        atomicAdd(reinterpret_cast<unsigned long long *>(acc), (unsigned long long)s);
}

hipError_t launch_debug_runsum(const BlockArgs &b, uint64_t nlo, uint64_t nhi, uint64_t ymax,
                               uint64_t L, uint64_t *acc, hipStream_t s)
{
    hipLaunchKernelGGL(k_debug_runsum, dim3(4096), dim3(256), 0, s, b, nlo, nhi, ymax, L, acc);
    return hipGetLastError();
}

__global__ void k_wide_plan(QueryArgs q)
{
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= q.w_n)
        return;
    const uint32_t qi = q.w_q[e];
    const uint64_t x = q.w_x[e];
    const U128 m = udiv128_bits(U128{q.q_n[qi], q.q_nhi[qi]}, x);
    const uint64_t k0 = q.q_L[qi] / x + 1;
    uint64_t K = (m.hi << 32) | (m.lo >> 32);
    const double md = (double)m.hi * 18446744073709551616.0 + (double)m.lo;
    const double kb = q.beta * sqrt(md);
    if (kb < 1.8e19 && (uint64_t)kb > K)
        K = (uint64_t)kb;
    if (K < k0 - 1)
        K = k0 - 1;
    const U128 Y = udiv128_bits(m, K + 1);
    q.w_mlo[e] = m.lo;
    q.w_mhi[e] = m.hi;
    q.w_K[e] = K;
    q.w_k0[e] = k0;
    q.w_Y[e] = Y.lo;  // < 2^32
}

hipError_t launch_wide_plan(const QueryArgs &q, hipStream_t s)
{
    if (q.w_n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_wide_plan, dim3((q.w_n + 63) / 64), dim3(64), 0, s, q);
    return hipGetLastError();
}

// Per entry: the k with floor(m/k) in [y1, y2] (k in [floor(m/(y2+1)) + 1,
// floor(m/y1)], within [k0, K]), and -K M(Y) when Y is in the block.
__global__ void k_wide_prep(QueryArgs q, BlockArgs b_in)
{
    const BlockArgs b = load_block(b_in);
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= q.w_n)
        return;
    const U128 m{q.w_mlo[e], q.w_mhi[e]};
    const uint64_t K = q.w_K[e], k0 = q.w_k0[e], Y = q.w_Y[e];
    const uint64_t y1e = b.y1 > 0 ? b.y1 : 1;
    const U128 lo = udiv128_bits(m, b.y2 + 1), hi = udiv128_bits(m, y1e);
    uint64_t klo = (lo.hi || lo.lo == ~0ull) ? ~0ull : lo.lo + 1;
    if (klo < k0)
        klo = k0;
    const uint64_t khi = (hi.hi || hi.lo > K) ? K : hi.lo;
    q.w_klo[e] = klo;
    q.w_khi[e] = khi;
    if (Y >= y1e && Y <= b.y2)
        q.S[q.w_g[e]] -= K * (uint64_t)M_at(b.words, Y - b.y1);
}

hipError_t launch_wide_prep(const QueryArgs &q, const BlockArgs &b, hipStream_t s)
{
    if (q.w_n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_wide_prep, dim3((q.w_n + 63) / 64), dim3(64), 0, s, q, b);
    return hipGetLastError();
}

// Per entry, over the whole grid: the explicit-k terms M(floor(m/k)) and the
// run-length terms floor(m/y) mu(y) for y in the block up to Y; one atomic
// per wave and entry into S.
constexpr uint32_t WIDE_WGS = 1024;

__global__ __launch_bounds__(256) void k_wide_update(QueryArgs q, BlockArgs b_in)
{
    const BlockArgs b = load_block(b_in);
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t y1e = b.y1 > 0 ? b.y1 : 1;
    for (uint32_t e = 0; e < q.w_n; ++e) {
        const uint64_t klo = q.w_klo[e], khi = q.w_khi[e];
        const uint64_t yhi = q.w_Y[e] < b.y2 ? q.w_Y[e] : b.y2;
        if (klo > khi && y1e > yhi)
            continue;
        const U128 m{q.w_mlo[e], q.w_mhi[e]};
        uint64_t acc = 0;
        if (klo <= khi) {
            const double md = (double)m.hi * 18446744073709551616.0 + (double)m.lo;
            for (uint64_t k = klo + gid; k <= khi; k += stride) {
                const uint64_t t = wide_quot_small(m, md, k);
                if (t >= b.y1 && t <= b.y2)  // always, by the choice of [klo, khi]
                    acc += (uint64_t)M_at(b.words, t - b.y1);
            }
        }
        for (uint64_t y = y1e + gid; y <= yhi; y += stride) {
            const uint64_t off = y - b.y1;
            const uint64_t rec = b.words[2 * (off >> 5)];
            const uint32_t bt = (uint32_t)(off & 31);
            const bool pos = (rec >> bt) & 1u, neg = (rec >> (32 + bt)) & 1u;
            if (pos || neg) {
                const uint64_t t = wide_quot_low(m, y);
                acc += pos ? t : 0 - t;
            }
        }
        acc = wave_sum_u64(acc);
        if (lane_id() == 0 && acc)
            atomicAdd(reinterpret_cast<unsigned long long *>(&q.S[q.w_g[e]]), acc);
    }
}

hipError_t launch_wide_update(const QueryArgs &q, const BlockArgs &b, hipStream_t s)
{
    if (q.w_n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_wide_update, dim3(WIDE_WGS), dim3(256), 0, s, q, b);
    return hipGetLastError();
}

hipError_t launch_update_prep(const QueryArgs &q, const BlockArgs &b, hipStream_t s, uint32_t wa,
                              uint32_t wb)
{
    const uint32_t grid = (q.ntiles + 3) / 4;
    hipLaunchKernelGGL(k_update_prep, dim3(grid), dim3(UPD_THREADS), 0, s, q, b, wa, wb);
    return hipGetLastError();
}

// In-place exclusive prefix of tile_items (ntiles entries); total at [ntiles].
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_items(QueryArgs q)
{
    __shared__ int64_t wsum[SCAN_THREADS / 64];
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (q.ntiles + SCAN_THREADS - 1) / SCAN_THREADS;
    const uint32_t t0 = tid * per;
    const uint32_t t1 = (t0 + per < q.ntiles) ? t0 + per : q.ntiles;
    int64_t local = 0;
    for (uint32_t t = t0; t < t1; ++t)
        local += (int64_t)q.tile_items[t];
    int64_t total;
    const int64_t ex = wg_exclusive_scan<SCAN_THREADS>(local, wsum, total);
    int64_t run = ex;
    for (uint32_t t = t0; t < t1; ++t) {
        const int64_t v = (int64_t)q.tile_items[t];
        q.tile_items[t] = (uint64_t)run;
        run += v;
    }
    if (tid == 0)
        q.tile_items[q.ntiles] = (uint64_t)total;
}

hipError_t launch_scan_items(const QueryArgs &q, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan_items, dim3(1), dim3(SCAN_THREADS), 0, s, q);
    return hipGetLastError();
}

// Largest t < ntiles with prefix[t] <= item (wave-parallel 64-ary search).
__device__ inline uint32_t find_tile(const uint64_t *__restrict__ prefix, uint32_t ntiles,
                                     uint64_t item)
{
    const uint32_t lane = lane_id();
    uint32_t lo = 0, hi = ntiles;
    while (hi - lo > 1) {
        const uint32_t stride = (hi - lo + 63) / 64;
        const uint32_t idx = lo + lane * stride;
        const bool ok = idx < hi && prefix[idx] <= item;
        const uint64_t bal = __ballot(ok);
        const uint32_t j = 63u - (uint32_t)__clzll((long long)bal);
        lo = lo + j * stride;
        const uint32_t nhi = lo + stride;
        hi = nhi < hi ? nhi : hi;
    }
    return lo;
}

// Exact quotients through fp64.  For m < 2^64 and 1 <= d < 2^32 with
// floor(m/d) < 2^32, the product (double)m * (1.0/d) carries three
// roundings of relative size 2^-53, so it lies within 2^-19.4 of m/d.
// When its fractional part is at least QEPS = 2^-19 away from an integer,
// its truncation is the exact floor; otherwise (rare) the lane recomputes
// the remainder in integers and corrects by one.
constexpr double QEPS = 1.0 / 524288.0;

__device__ inline double readlane_f64(double v, uint32_t lane)
{
    return __longlong_as_double((long long)readlane_u64((uint64_t)__double_as_longlong(v), lane));
}

// exact floor(m/d) from the truncated estimate t (|t - m/d| < 1)
__device__ inline uint64_t fix_quotient(uint64_t m, uint64_t d, double t)
{
    uint64_t qv = (uint64_t)t;
    const int64_t r = (int64_t)(m - qv * d);
    if (r < 0)
        qv -= 1;
    else if ((uint64_t)r >= d)
        qv += 1;
    return qv;
}

constexpr int RL_XS = 16;
constexpr uint32_t RL_ENT_SPAN = 4096;  // y per compacted sub-chunk
constexpr uint32_t RL_ENT_CAP = 3072;   // 1024 of any 4096 consecutive y are multiples of 4

// Below this m the rounded-up reciprocal gives exact floors with no test.
constexpr double RL_M_EXACT = 281474976710656.0;  // 2^48

// 1/y within one unit in the last place: the hardware estimate refined by
// two fused Newton steps (e = 1 - y r, r += r e).  From an estimate within
// 2^-20 the first step leaves a relative error near 2^-40, the second only
// its final rounding (half a unit) plus terms near 2^-80.
__device__ inline double rcp_1ulp(double y)
{
    double r = __builtin_amdgcn_rcp(y);
    double e = fma(-y, r, 1.0);
    r = fma(r, e, r);
    e = fma(-y, r, 1.0);
    return fma(r, e, r);
}

// 1/k raised by 2^-50 of itself: rcp_1ulp whose second Newton step aims at
// (1 + 2^-50)/k.  With r1 = (1 - e1)/k after the first step (|e1| near
// 2^-40), e = RN(1 + 2^-50 - k r1) = (2^-50 + e1)(1 + h) and
// r' = RN(r1 + r1 e) = (1/k)(1 + 2^-50 - e1^2 - 2^-50 e1 + (2^-50 + e1) h
// (1 - e1))(1 + h'), |h|, |h'| <= 2^-53: r' = (1/k)(1 + b) with b within
// 2^-53 + 2^-79 of 2^-50, i.e. in [2^-50.2, 2^-49.8].  For m < 2^48 the
// product m * rcp_up(k) rounded once then lies in [m/k, (m/k)(1 + 2^-49.6)],
// whose floor is floor(m/k) (see rl_pass).
constexpr double RCP_UP_ONE = 1.0000000000000008881784197001;  // 1 + 2^-50
static_assert(RCP_UP_ONE == 1.0 + 0x1p-50, "1 + 2^-50 exactly");
__device__ inline double rcp_up(double k)
{
    double r = __builtin_amdgcn_rcp(k);
    double e = fma(-k, r, 1.0);
    r = fma(r, e, r);
    e = fma(-k, r, RCP_UP_ONE);
    return fma(r, e, r);
}

// One pass of RL_XS x (m as fp64 in mf, NaN past the tile's end) over the
// compacted entries.
// * FAST (every m < 2^48, every y <= Y): r' = rcp_up(y) lies in
//   [(1/y)(1 + 2^-50.2), (1/y)(1 + 2^-49.8)], so qd = RN(m r') lies in
//   [m/y, (m/y)(1 + 2^-49.6)]: never below m/y, and above the next integer
//   only if m/y were within (m/y) 2^-49.6 < 1/y of it, which m mod y >= 0
//   rules out.  floor(qd) =
//   floor(m/y) exactly: three fp64 ops per pair.
// * otherwise: qh = m/y - 1/2 rounded once (fma); t = rint(qh) is
//   floor(m/y) unless qh lies within QEPS of a half-integer, which the
//   running max of |qh - t| detects; such entries redo the RL_XS pairs with
//   the integer fix-up.  With YCHECK, pairs with y > Y_x are skipped
//   (sub-chunks that straddle some x's Y); *cnt counts the pairs taken.
// * FAST23 (as FAST, and every quotient of the pass below 2^23): with the
//   same r', fma(m, r', 2^52 - 1/2) is exactly 2^52 + floor(m/y), since the
//   exact m r' + 2^52 - 1/2 lies strictly between 2^52 + q - 1/2 and
//   2^52 + q + 1/2 and one rounding takes it to the integer grid of
//   [2^52, 2^53); the low word of the result is q, added with its sign by a
//   24-bit multiply-add into 32-bit sums (at most 48 entries per lane and
//   pass, |sum| < 2^29): two ops per pair.
enum { RL_FAST = 0, RL_NEAR = 1, RL_NEAR_Y = 2, RL_FAST23 = 3 };
constexpr double RL_MAGIC = 4503599627370495.5;  // 2^52 - 1/2
constexpr double RL_Q23 = 8388608.0;             // 2^23

template <int MODE>
__device__ inline void rl_pass(const uint16_t *ent, uint32_t total, uint32_t wb0,
                               const double (&mf)[RL_XS], const uint32_t (&Yv)[RL_XS],
                               const uint64_t *xm, double (&acc)[RL_XS], uint32_t *cnt)
{
    constexpr bool YCHECK = MODE == RL_NEAR_Y;
    const uint32_t lane = lane_id();
    int acc32[RL_XS];
#pragma unroll
    for (int i = 0; i < RL_XS; ++i)
        acc32[i] = 0;
    for (uint32_t t = lane; t < total; t += 64) {
        const uint32_t e = ent[t];
        const uint32_t y = wb0 + (e & 0x0FFFu);
        const double sg = (e & 0x8000u) ? -1.0 : 1.0;
        if (MODE == RL_FAST) {
            const double ru = rcp_up((double)y);
#pragma unroll
            for (int i = 0; i < RL_XS; ++i)
                acc[i] = fma(sg, floor(mf[i] * ru), acc[i]);
            continue;
        }
        if (MODE == RL_FAST23) {
            const double ru = rcp_up((double)y);
            int si = (e & 0x8000u) ? -1 : 1;
            // opaque: a known +-1 factor is otherwise expanded into a
            // conditional negation (four ops instead of one multiply-add)
            __asm__ volatile("" : "+v"(si));
#pragma unroll
            for (int i = 0; i < RL_XS; ++i) {
                // NaN m (past the tile) gives the canonical NaN: low word 0
                const double t = fma(mf[i], ru, RL_MAGIC);
                acc32[i] += __mul24((int)(uint32_t)__double_as_longlong(t), si);
            }
            continue;
        }
        const double r = 1.0 / (double)y;
        double dmax = 0.0;
#pragma unroll
        for (int i = 0; i < RL_XS; ++i) {
            if (YCHECK && y > Yv[i])
                continue;
            const double qh = fma(mf[i], r, -0.5);
            const double tq = rint(qh);
            acc[i] = fma(sg, tq, acc[i]);
            dmax = fmax(dmax, fabs(qh - tq));
            if (YCHECK)
                *cnt += 1;
        }
        if (dmax > 0.5 - QEPS) {
            // opaque copy: recompute here rather than keep RL_XS values live
            double r2 = r;
            __asm__ volatile("" : "+v"(r2));
#pragma unroll
            for (int i = 0; i < RL_XS; ++i) {
                if (YCHECK && y > Yv[i])
                    continue;
                const double qh = fma(mf[i], r2, -0.5);
                const double tq = rint(qh);
                if (fabs(qh - tq) > 0.5 - QEPS) {
                    const uint64_t exact = fix_quotient(xm[i], y, tq);
                    acc[i] = fma(sg, (double)(int64_t)(exact - (uint64_t)tq), acc[i]);
                }
            }
        }
    }
    if (MODE == RL_FAST23) {
#pragma unroll
        for (int i = 0; i < RL_XS; ++i)
            acc[i] = (double)acc32[i];
    }
}

// Sum of each of RL_XS = 16 values over the wave, by halving exchanges:
// after the xor-32/16/8/4 steps lane l holds a partial sum of value
// (l >> 2) only, and the xor-2/1 steps complete it on all four lanes of
// each quad (17 exchanges instead of 16 full reductions).
__device__ inline double wave_multi_sum16(double (&a)[RL_XS])
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int h = 8; h >= 1; h >>= 1) {
        const int o = h * 4;  // 32, 16, 8, 4
        const bool up = (lane & (uint32_t)o) != 0;
#pragma unroll
        for (int j = 0; j < h; ++j) {
            const double send = up ? a[j] : a[j + h];
            const double keep = up ? a[j + h] : a[j];
            a[j] = keep + __shfl_xor(send, o, 64);
        }
    }
    double v = a[0];
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 1, 64);
    return v;
}

// The FAST23 pass (see rl_pass) over 32 x at once, for sub-chunks where
// every x of the tile qualifies: one reciprocal and entry decode per 32
// pairs instead of per 16.
constexpr int RL_XS2 = 32;

__device__ inline void rl_pass_fast23_32(const uint16_t *ent, uint32_t total, uint32_t wb0,
                                         const double (&mf)[RL_XS2], int (&acc32)[RL_XS2])
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int i = 0; i < RL_XS2; ++i)
        acc32[i] = 0;
    for (uint32_t t = lane; t < total; t += 64) {
        const uint32_t e = ent[t];
        const double ru = rcp_up((double)(wb0 + (e & 0x0FFFu)));
        int si = (e & 0x8000u) ? -1 : 1;
        __asm__ volatile("" : "+v"(si));  // keep the multiply-add (see rl_pass)
#pragma unroll
        for (int i = 0; i < RL_XS2; ++i) {
            const double tq = fma(mf[i], ru, RL_MAGIC);
            acc32[i] += __mul24((int)(uint32_t)__double_as_longlong(tq), si);
        }
    }
}

// Sum of each of 32 int values over the wave, by halving exchanges: after
// the xor-32/16/8/4/2 steps lane l holds a partial sum of value l >> 1 only,
// and the xor-1 step completes it on both lanes of each pair.
__device__ inline int wave_multi_sum32_i(int (&a)[RL_XS2])
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int h = 16; h >= 1; h >>= 1) {
        const int o = h * 2;  // 32, 16, 8, 4, 2
        const bool up = (lane & (uint32_t)o) != 0;
#pragma unroll
        for (int j = 0; j < h; ++j) {
            const int send = up ? a[j] : a[j + h];
            const int keep = up ? a[j + h] : a[j];
            a[j] = keep + __shfl_xor(send, o, 64);
        }
    }
    int v = a[0];
    v += __shfl_xor(v, 1, 64);
    return v;
}

// Run-length part, lanes over y.  The item's y range is taken in sub-chunks
// of 4096 aligned y: the squarefree y of a sub-chunk are compacted into LDS
// (12-bit offset | sign << 15) and each lane takes every 64th entry against
// RL_XS x of the tile at a time (m_x uniform), i.e. RL_XS independent
// quotient chains per lane and entry.  Per-x sums stay in registers (lane l
// holds x (l >> 2) + 16 (l & 3)) and leave with one 64-lane atomic per
// item.  Requires every quotient below 2^32 (y > m/2^32 for every x of the
// tile) and y < 2^32.
__device__ inline void mu_item_lanes(const QueryArgs &q, const BlockArgs &b, uint32_t tile,
                                     uint64_t cs, uint64_t ce, uint16_t *ent)
{
    const uint32_t lane = lane_id();
    const uint32_t nx = __builtin_amdgcn_readfirstlane(q.tile_nx[tile]);
    const uint64_t g0 = uniform_u64(q.tile_g0[tile]);
    // lane l sums x (l >> 2) + 16 (l & 3) of the tile
    const uint32_t qd = lane & 3u, xi = (lane >> 2) + 16u * qd;
    double mine = 0.0;
    uint64_t nq = 0;
    // the tile's largest m and smallest Y (32-x FAST23 passes need every x
    // to qualify)
    uint64_t t_mmax, t_ymin;
    {
        const bool ok = lane < nx;
        t_mmax = uniform_u64(wave_max_u64(ok ? q.x_m[g0 + lane] : 0ull));
        t_ymin = uniform_u64(wave_min_u64(ok ? q.x_Y[g0 + lane] : ~0ull));
    }
    for (uint64_t sb = cs & ~63ull; sb <= ce; sb += RL_ENT_SPAN) {
        const uint64_t ss = sb > cs ? sb : cs;
        const uint64_t se = (ce - sb) < RL_ENT_SPAN - 1 ? ce : sb + RL_ENT_SPAN - 1;
        const uint32_t nw = (uint32_t)((se - sb) >> 6) + 1;  // <= 64
        uint64_t bits = 0, ngw = 0;
        if (lane < nw) {
            const uint64_t wbase = sb + 64ull * lane;
            uint64_t nzm;
            word_masks(b.words, (wbase - b.y1) >> 6, nzm, ngw);
            const uint32_t lob = wbase < ss ? (uint32_t)(ss - wbase) : 0u;
            const uint32_t hib = (se - wbase) < 63 ? (uint32_t)(se - wbase) : 63u;
            bits = nzm & (~0ull << lob) & ((2ull << hib) - 1ull);
        }
        const uint32_t cnt = (uint32_t)__popcll(bits);
        uint32_t incl = cnt;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(incl, o, 64);
            if (lane >= (uint32_t)o)
                incl += t;
        }
        const uint32_t total = __builtin_amdgcn_readlane(incl, 63);
        // the previous sub-chunk's readers are done with ent
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        uint32_t pos = incl - cnt;
        while (bits) {
            const uint32_t bt = (uint32_t)__builtin_ctzll(bits);
            bits &= bits - 1;
            ent[pos++] = (uint16_t)((lane * 64 + bt) | (uint32_t)(((ngw >> bt) & 1ull) << 15));
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();

        if (q.rl_fast && se <= t_ymin && (double)t_mmax < RL_M_EXACT &&
            (double)t_mmax < RL_Q23 * (double)ss) {
            // two passes of 32 x; lane l then holds x 32 p + (l >> 1), and the
            // lane that sums x in the 16-x layout takes it over
#pragma unroll 1
            for (uint32_t p = 0; p < 2; ++p) {
                const uint32_t xs = p * RL_XS2;
                if (xs >= nx)
                    break;
                double mf[RL_XS2];
                int acc32[RL_XS2];
#pragma unroll
                for (int i = 0; i < RL_XS2; ++i) {
                    const bool ok = xs + (uint32_t)i < nx;
                    const uint64_t mi = ok ? uniform_u64(q.x_m[g0 + xs + i]) : 0;
                    // NaN past the tile's end: the result's low word is 0
                    mf[i] = ok ? (double)mi : __longlong_as_double(0x7ff8000000000000ll);
                }
                rl_pass_fast23_32(ent, total, (uint32_t)sb, mf, acc32);
                const int v = wave_multi_sum32_i(acc32);
                const int w = __shfl(v, (int)(2u * (xi - xs)) & 63, 64);
                if ((xi >> 5) == p)
                    mine += (double)w;
                const uint32_t nxs = (nx - xs) < (uint32_t)RL_XS2 ? nx - xs : (uint32_t)RL_XS2;
                nq += lane == 0 ? (uint64_t)total * nxs : 0;
            }
            continue;
        }

#pragma unroll 1
        for (uint32_t p = 0; p < 4; ++p) {
            const uint32_t xs = p * RL_XS;
            if (xs >= nx)
                break;
            const uint32_t nxs = (nx - xs) < (uint32_t)RL_XS ? nx - xs : (uint32_t)RL_XS;
            double mf[RL_XS], acc[RL_XS];
            uint32_t Yv[RL_XS];
            uint32_t ymin = ~0u;
            uint64_t mmax = 0;
#pragma unroll
            for (int i = 0; i < RL_XS; ++i) {
                const bool ok = (uint32_t)i < nxs;
                const uint64_t mi = ok ? uniform_u64(q.x_m[g0 + xs + i]) : 0;
                Yv[i] = ok ? (uint32_t)uniform_u64(q.x_Y[g0 + xs + i]) : 0u;
                // NaN past the tile's end: never near a half-integer, never summed
                mf[i] = ok ? (double)mi : __longlong_as_double(0x7ff8000000000000ll);
                acc[i] = 0.0;
                if (ok && Yv[i] < ymin)
                    ymin = Yv[i];
                mmax = mi > mmax ? mi : mmax;
            }
            const uint64_t *xm = q.x_m + g0 + xs;
            if (se > ymin) {  // some y of the sub-chunk exceeds some x's Y
                uint32_t c = 0;
                rl_pass<RL_NEAR_Y>(ent, total, (uint32_t)sb, mf, Yv, xm, acc, &c);
                nq += c;
            } else {
                if (q.rl_fast && (double)mmax < RL_M_EXACT && (double)mmax < RL_Q23 * (double)ss)
                    rl_pass<RL_FAST23>(ent, total, (uint32_t)sb, mf, Yv, xm, acc, nullptr);
                else if (q.rl_fast && (double)mmax < RL_M_EXACT)
                    rl_pass<RL_FAST>(ent, total, (uint32_t)sb, mf, Yv, xm, acc, nullptr);
                else
                    rl_pass<RL_NEAR>(ent, total, (uint32_t)sb, mf, Yv, xm, acc, nullptr);
                nq += lane == 0 ? (uint64_t)total * nxs : 0;
            }
            // NaN sums of absent x stay on lanes that never write them
            const double v = wave_multi_sum16(acc);
            if (qd == p)
                mine += v;
        }
    }
    if (xi < nx)
        atomicAdd((unsigned long long *)&q.S[g0 + xi], (unsigned long long)(int64_t)mine);
    nq = wave_sum_u64(nq);
    if (lane == 0)
        atomicAdd((unsigned long long *)&q.pair_stats[2], (unsigned long long)nq);
}

// Run-length part of one (tile, y-chunk) item:
//   S[x] += sum_{y in chunk, y <= Y_x, mu(y) != 0} mu(y) floor(m_x / y).
// y is uniform across the wave (lane = x): the mask words come from scalar
// loads, and per 64-y word each lane computes one divisor's constants (1/y
// for the fp64 path, the Granlund-Montgomery multiplier for the integer
// path), which readlane broadcasts.
__device__ inline void mu_item(const QueryArgs &q, const BlockArgs &b, uint32_t tile, uint64_t c,
                               uint16_t *ent)
{
    const uint32_t lane = lane_id();
    const uint32_t nx = q.tile_nx[tile];
    const uint64_t g = q.tile_g0[tile] + lane;
    const bool valid = lane < nx;
    const uint64_t m = valid ? q.x_m[g] : 0;
    const uint64_t Y = valid ? q.x_Y[g] : 0;
    // m as fp64; NaN on lanes past the tile's end, so their near-integer
    // test below never fires (they never write S)
    const double mfq = valid ? (double)m : __longlong_as_double(0x7ff8000000000000ll);
    // y > qbig => every quotient of the tile is below 2^32
    const uint64_t qbig = uniform_u64(wave_max_u64(m)) >> 32;
    const uint64_t ymin = uniform_u64(wave_min_u64(valid ? Y : ~0ull));
    const uint64_t y1e = b.y1 > 0 ? b.y1 : 1;
    const uint64_t tymax = uniform_u64(q.tile_ymax[tile]);
    const uint64_t yb_t = tymax < b.y2 ? tymax : b.y2;
    const uint64_t yal = y1e & ~63ull;
    uint64_t cs = yal + c * q.ychunk;
    uint64_t ce = cs + q.ychunk - 1;
    if (ce > yb_t)
        ce = yb_t;
    if (cs < y1e)
        cs = y1e;
    if (ent && cs > qbig && cs <= ce && ce < (1ull << 32)) {
        mu_item_lanes(q, b, tile, cs, ce, ent);
        return;
    }
    uint64_t acc = 0, nq = 0;
    double accf = 0.0;  // integer-valued, |accf| < ychunk * 2^32 <= 2^52
    for (uint64_t wbase = cs & ~63ull; wbase <= ce; wbase += 64) {
        const uint64_t woff = (wbase - b.y1) >> 6;
        uint64_t nzv, ngv;
        word_masks(b.words, woff, nzv, ngv);
        const uint64_t nz = uniform_u64(nzv);
        const uint64_t ng = uniform_u64(ngv);
        const uint32_t lob = wbase < cs ? (uint32_t)(cs - wbase) : 0u;
        const uint32_t hib = (ce - wbase) < 63 ? (uint32_t)(ce - wbase) : 63u;
        uint64_t bits = nz & (~0ull << lob) & ((2ull << hib) - 1ull);
        if (bits == 0)
            continue;
        // quotients this lane takes in this word (bits with y <= Y)
        if (Y >= wbase)
            nq += (Y - wbase >= 63) ? __popcll(bits) : __popcll(bits & ((2ull << (Y - wbase)) - 1ull));
        if (wbase > qbig) {
            const double rl = 1.0 / (double)(wbase + lane);
            if (wbase + 63 <= ymin) {
                // every lane takes every y of the word; mu = +1 bits, then -1
                uint64_t pos = bits & ~ng, neg = bits & ng;
                while (pos) {
                    const uint32_t bt = (uint32_t)__builtin_ctzll(pos);
                    pos &= pos - 1;
                    const double qd = mfq * readlane_f64(rl, bt);
                    const double t = trunc(qd);
                    accf += t;
                    if (fabs(qd - t - 0.5) > 0.5 - QEPS)
                        accf += (double)(int64_t)(fix_quotient(m, wbase + bt, t) - (uint64_t)t);
                }
                while (neg) {
                    const uint32_t bt = (uint32_t)__builtin_ctzll(neg);
                    neg &= neg - 1;
                    const double qd = mfq * readlane_f64(rl, bt);
                    const double t = trunc(qd);
                    accf -= t;
                    if (fabs(qd - t - 0.5) > 0.5 - QEPS)
                        accf -= (double)(int64_t)(fix_quotient(m, wbase + bt, t) - (uint64_t)t);
                }
            } else {
                while (bits) {
                    const uint32_t bt = (uint32_t)__builtin_ctzll(bits);
                    bits &= bits - 1;
                    const uint64_t y = wbase + bt;
                    const double qd = mfq * readlane_f64(rl, bt);
                    if (y <= Y) {
                        double t = trunc(qd);
                        if (fabs(qd - t - 0.5) > 0.5 - QEPS)
                            t = (double)fix_quotient(m, y, t);
                        accf += ((ng >> bt) & 1ull) ? -t : t;
                    }
                }
            }
        } else {
            // quotients may reach 2^32: Granlund-Montgomery integer path
            uint64_t mul;
            uint32_t sh1, sh2;
            gm_magic((uint32_t)(wbase + lane), mul, sh1, sh2);
            while (bits) {
                const uint32_t bt = (uint32_t)__builtin_ctzll(bits);
                bits &= bits - 1;
                const uint64_t y = wbase + bt;
                const uint64_t mg = readlane_u64(mul, bt);
                const uint32_t s1 = __builtin_amdgcn_readlane(sh1, bt);
                const uint32_t s2 = __builtin_amdgcn_readlane(sh2, bt);
                const uint64_t qv = gm_div(m, mg, s1, s2);
                if (y <= Y) {
                    if ((ng >> bt) & 1ull)
                        acc -= qv;
                    else
                        acc += qv;
                }
            }
        }
    }
    acc += (uint64_t)(int64_t)accf;
    if (valid)
        atomicAdd((unsigned long long *)&q.S[g], (unsigned long long)acc);
    nq = wave_sum_u64(nq);
    if (lane == 0)
        atomicAdd((unsigned long long *)&q.pair_stats[2], (unsigned long long)nq);
}

// exact floor(m / k) for any k >= 1 from an fp64 estimate and integer
// correction steps (one step suffices while the quotient is below 2^50)
// floor(m/k) from an fp64 estimate t of m/k: the remainder is corrected in
// integers; the estimate is off by at most t * 2^-50 + 1, so the loops end
// after a step or two for any quotient the sweep produces.
__device__ inline uint64_t fix_quotient_any(uint64_t m, uint64_t k, double t)
{
    uint64_t qv = (uint64_t)t;
    int64_t r = (int64_t)(m - qv * k);
    while (r < 0) {
        qv -= 1;
        r += (int64_t)k;
    }
    while ((uint64_t)r >= k) {
        qv += 1;
        r -= (int64_t)k;
    }
    return qv;
}

// M(y1 + off) for K_UNROLL offsets at once: every record is requested
// before any is used, so each lane keeps K_UNROLL gathers in flight (the
// explicit k part is bound by gather latency, not by arithmetic).
constexpr int K_UNROLL = 4;

__device__ inline uint64_t M_sum_masked(const uint64_t *__restrict__ words,
                                        const uint64_t (&off)[K_UNROLL],
                                        const bool (&act)[K_UNROLL])
{
    ulonglong2 rec[K_UNROLL];
#pragma unroll
    for (int u = 0; u < K_UNROLL; ++u)
        rec[u] = *reinterpret_cast<const ulonglong2 *>(words + 2 * (off[u] >> 5));
    uint64_t s = 0;
#pragma unroll
    for (int u = 0; u < K_UNROLL; ++u) {
        const uint32_t lm = (2u << (uint32_t)(off[u] & 31)) - 1u;
        const uint64_t v = rec[u].y + (uint64_t)__popc((uint32_t)rec[u].x & lm) -
                           (uint64_t)__popc((uint32_t)(rec[u].x >> 32) & lm);
        s += act[u] ? v : 0ull;
    }
    return s;
}

// The same for block offsets off < 2^31 in 32-bit arithmetic: the record's
// byte offset is (off >> 5) * 16 = (off >> 1) & ~15, the mu sums within the
// record are added in 32 bits and the records' M in 64, and an inactive
// lane masks nothing in and adds no record.
__device__ inline uint64_t M_sum_masked32(const uint64_t *__restrict__ words,
                                          const uint32_t (&off)[K_UNROLL],
                                          const bool (&act)[K_UNROLL])
{
    const char *base = reinterpret_cast<const char *>(words);
    ulonglong2 rec[K_UNROLL];
#pragma unroll
    for (int u = 0; u < K_UNROLL; ++u)
        rec[u] = *reinterpret_cast<const ulonglong2 *>(base + ((off[u] >> 1) & ~15u));
    uint64_t s = 0;
    int32_t d = 0;
#pragma unroll
    for (int u = 0; u < K_UNROLL; ++u) {
        const uint32_t lm = act[u] ? (2u << (off[u] & 31)) - 1u : 0u;
        d += __popc((uint32_t)rec[u].x & lm) - __popc((uint32_t)(rec[u].x >> 32) & lm);
        s += act[u] ? rec[u].y : 0ull;
    }
    return s + (uint64_t)(int64_t)d;
}

// Explicit k part of one (tile, k-chunk) item with lanes as an 8 x 8 grid:
// lane = 8 xi + kj takes x = 8 g + xi of x-group g and k = kk + kj, so one
// gather instruction covers 8 neighbouring x and 8 neighbouring k, whose
// quotients floor(m/k) lie closer together than 64 x at one k or 64 k at
// one x (fewer cache lines per gather).  The reciprocals of the chunk's k
// are computed once per sub-chunk into LDS; per-x sums are reduced over the
// 8 k-lanes and leave with one 64-lane atomic per item.
constexpr uint32_t K2D_SUB = 512;  // k per reciprocal sub-chunk (4 KB of LDS)


// Record loads in flight per lane and batch of the walk below (8 x 8
// lanes, 16 batches: 128 consecutive k per x in flight).  Measured at
// M(10^16): 16 beats 8 by 2%; issuing the next batch before summing the
// current one (two alternating batches) was slower (registers spilled).
constexpr int K2F_UNROLL = 16;
// A y offset that no lane of a block can have: its record byte offset
// (0x7FFFFFF0) lies past every block's records, where a buffer load reads
// zeros (empty masks, M = 0), and its shift below is 0.
constexpr uint32_t OFF_NONE = ~0u;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Record sources of the walk below, by y offset from the base the offsets
// are taken from (OFF_NONE: the empty record).
// Global: buffer loads whose range is the block's records (a load past it
// reads zeros).
struct RecGlobal {
    __amdgpu_buffer_rsrc_t rs;
    __device__ u32x4 operator()(uint32_t off) const
    {
        return __builtin_amdgcn_raw_buffer_load_b128(rs, (off >> 1) & ~15u, 0, 0);
    }
};
// LDS: a window of EKW_REC records followed by one empty record.  Offsets
// are below 32 EKW_REC (a pair's quotient lies in the window) or equal to
// EKW_NONE, which names the empty record.
struct RecLds {
    const u32x4 *win;
    __device__ u32x4 operator()(uint32_t off) const { return win[off >> 5]; }
};

// One batch of the walk: U pairs per lane, k = sb + i0 + 8u.
template <int U>
struct K2Batch {
    uint32_t off[U];
    u32x4 rec[U];
};

template <int U, class Src>
__device__ inline void k2_issue(K2Batch<U> &t, const Src &src, const double *rk, uint32_t i0,
                                uint32_t lo_r, uint32_t cnt, double mf, double ny1)
{
    const uint32_t d0 = i0 - lo_r;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t o = (uint32_t)fma(mf, rk[i0 + 8 * u], ny1);
        t.off[u] = d0 + 8u * u < cnt ? o : OFF_NONE;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
        t.rec[u] = src(t.off[u]);
}

// acc + popcount(x) in one op (the compiler counts into zero and adds the
// counts with three-input adds: one op more per pair)
__device__ inline uint32_t popc_add(uint32_t x, uint32_t acc)
{
    uint32_t r;
    __asm__("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

template <int U>
__device__ inline void k2_consume(const K2Batch<U> &t, uint32_t &dp, uint32_t &dn, uint64_t &ms)
{
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t sh = ~t.off[u] & 31u;
        dp = popc_add(t.rec[u].x << sh, dp);
        dn = popc_add(t.rec[u].y << sh, dn);
        ms += (uint64_t)t.rec[u].z | ((uint64_t)t.rec[u].w << 32);
    }
}

// The pairs k in [lo, hi] (this lane's x; sb <= lo) of one group of eight x
// over the reciprocal table rk of the sub-chunk from sb: the group walks the
// union of its lanes' ranges, 8 x 8 lanes, batches of U pairs per lane.
template <int U, class Src>
__device__ inline void k2_walk(const Src &src, const double *rk, uint64_t sb, uint32_t kj,
                               double mf, double ny1, uint64_t lo, uint64_t hi, uint32_t &dp,
                               uint32_t &dn, uint64_t &ms)
{
    constexpr uint32_t STEP = 8 * U;
    const bool has = lo <= hi;
    const uint64_t glo = uniform_u64(wave_min_u64(has ? lo : ~0ull));
    const uint64_t ghi = uniform_u64(wave_max_u64(has ? hi : 0ull));
    if (glo > ghi)
        return;
    // pair k = sb + i is active when (i - lo_r) mod 2^32 < cnt
    const uint32_t lo_r = (uint32_t)(lo - sb);
    const uint32_t cnt = has ? (uint32_t)(hi - lo) + 1u : 0u;
    // indices read reach (ghi - sb) + STEP - 1 < K2D_SUB + STEP: inside the
    // table's slice; values past the filled ones are never used
    const uint32_t ilo = (uint32_t)(glo - sb), ihi = (uint32_t)(ghi - sb);
    for (uint32_t kr = ilo; kr <= ihi; kr += STEP) {
        K2Batch<U> t;
        k2_issue<U>(t, src, rk, kr + kj, lo_r, cnt, mf, ny1);
        k2_consume<U>(t, dp, dn, ms);
    }
}


// The 8 x 8 walk of k_item_2d for tiles whose m are all below 2^48, with no
// branch per pair.  Lane l brings m, k_lo and k_hi of the tile's x l (taken
// once per item; lanes past the tile hold an empty range), and each group of
// eight x reads them by lane exchange.
// * y - y1 = trunc(fma(m, rcp_up(k), -y1)).  In a block from y1 = 0 this is
//   the product above.  From y1 > 0 with y2 - y1 < y1: active pairs have
//   k <= m/y1, so the product's excess over floor(m/k) stays below the next
//   integer by more than (1/k)(1 - m 2^-49.8) >= 0.67 y1/m, while the one
//   rounding of the fused result (< 2^31 = y2 - y1 + 1 <= y1) moves it by at
//   most (y2 - y1 + 1) 2^-53 < 0.67 y1 / m; rounding never goes below the
//   integer floor(m/k) - y1 either, since the exact value exceeds it.
// * Records come through buffer loads whose range is the block's records;
//   lanes outside their x's k range take OFF_NONE and add nothing.
// * The mu sum up to y within its record is the population count of each
//   mask shifted left by 31 - (y mod 32) (the low five bits of ~off).
// * With a band (wa < wb), each x's band k are left out (two walks, below
//   and above them).
__device__ inline void k_item_2d_fast(const QueryArgs &q, const BlockArgs &b, uint32_t tile,
                                      uint64_t kb, uint64_t ke, double *rk, uint64_t m_l,
                                      uint64_t klo_l, uint64_t khi_l, uint32_t wa, uint32_t wb)
{
    const uint32_t lane = lane_id(), xi = lane >> 3, kj = lane & 7u;
    const uint32_t nx = __builtin_amdgcn_readfirstlane(q.tile_nx[tile]);
    const uint64_t g0 = uniform_u64(q.tile_g0[tile]);
    const uint32_t rec_bytes = ((uint32_t)((b.y2 - b.y1) >> 5) + 1u) * 16u;
    const RecGlobal src{
        __builtin_amdgcn_make_buffer_rsrc(b.words, (short)0, (int)rec_bytes, 0x00020000)};
    const double ny1 = -(double)b.y1;
    const bool band = wa < wb;
    uint64_t mine = 0;  // lane holds x = 8 kj + xi
    for (uint64_t sb = kb; sb <= ke; sb += K2D_SUB) {
        const uint64_t se = (ke - sb) < K2D_SUB - 1 ? ke : sb + K2D_SUB - 1;
        const uint32_t ns = (uint32_t)(se - sb) + 1;
        // the previous sub-chunk's readers are done with rk
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (uint32_t i = lane; i < ns; i += 64)
            rk[i] = rcp_up((double)(sb + i));
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll 1
        for (uint32_t g = 0; g < 8; ++g) {
            const int sl = (int)(8 * g + xi);
            const uint64_t m = __shfl(m_l, sl, 64);
            uint64_t lo = __shfl(klo_l, sl, 64);
            uint64_t hi = __shfl(khi_l, sl, 64);
            lo = lo > sb ? lo : sb;
            hi = hi < se ? hi : se;
            const double mf = (double)m;
            uint64_t ms = 0;
            uint32_t dp = 0, dn = 0;
            if (band) {
                const uint64_t hl = (m >> wb) + 1, hh = m >> wa;  // the band's k
                k2_walk<K2F_UNROLL>(src, rk, sb, kj, mf, ny1, lo, hi < hl - 1 ? hi : hl - 1, dp,
                                    dn, ms);
                k2_walk<K2F_UNROLL>(src, rk, sb, kj, mf, ny1, lo > hh + 1 ? lo : hh + 1, hi, dp,
                                    dn, ms);
            } else {
                k2_walk<K2F_UNROLL>(src, rk, sb, kj, mf, ny1, lo, hi, dp, dn, ms);
            }
            uint64_t acc = ms + (uint64_t)(int64_t)(int32_t)(dp - dn);
            acc += __shfl_xor(acc, 1, 64);
            acc += __shfl_xor(acc, 2, 64);
            acc += __shfl_xor(acc, 4, 64);
            if (kj == g)
                mine += acc;
        }
    }
    const uint32_t xo = 8 * kj + xi;
    if (xo < nx)
        atomicAdd((unsigned long long *)&q.S[g0 + xo], (unsigned long long)mine);
}

__device__ inline void k_item_2d(const QueryArgs &q, const BlockArgs &b, uint32_t tile,
                                 uint64_t c, double *rk, uint32_t wa, uint32_t wb)
{
    const uint32_t lane = lane_id(), xi = lane >> 3, kj = lane & 7u;
    const uint32_t nx = __builtin_amdgcn_readfirstlane(q.tile_nx[tile]);
    const uint64_t g0 = uniform_u64(q.tile_g0[tile]);
    const uint64_t tklo = uniform_u64(q.tile_klo[tile]);
    const uint64_t tkhi = uniform_u64(q.tile_khi[tile]);
    uint64_t kb = tklo + c * q.kchunk;
    uint64_t ke = (tkhi - kb) < (uint64_t)q.kchunk - 1 ? tkhi : kb + q.kchunk - 1;
    if (q.rl_fast && (b.y1 == 0 || b.y2 - b.y1 < b.y1)) {
        // lane l: the tile's x l (an empty k range past the tile)
        uint64_t m_l = 0, klo_l = 1, khi_l = 0;
        if (lane < nx) {
            m_l = q.x_m[g0 + lane];
            klo_l = q.x_klo[g0 + lane];
            khi_l = q.x_khi[g0 + lane];
        }
        if (uniform_u64(wave_max_u64(m_l)) < (1ull << 48)) {
            if (wa < wb) {  // a band tile: its chunks skip the gap the band leaves
                uint64_t amax, bmin;
                band_gap(m_l, klo_l, khi_l, wa, wb, amax, bmin);
                const KChunks ch = k_chunks(tklo, tkhi, q.kchunk, true, amax, bmin);
                if (c < ch.n_a) {
                    ke = (ch.aend - kb) < (uint64_t)q.kchunk - 1 ? ch.aend : kb + q.kchunk - 1;
                } else {
                    kb = ch.bmin + (c - ch.n_a) * q.kchunk;
                    ke = (tkhi - kb) < (uint64_t)q.kchunk - 1 ? tkhi : kb + q.kchunk - 1;
                }
            }
            k_item_2d_fast(q, b, tile, kb, ke, rk, m_l, klo_l, khi_l, wa, wb);
            return;
        }
    }
    uint64_t mine = 0;  // lane holds x = 8 kj + xi
    for (uint64_t sb = kb; sb <= ke; sb += K2D_SUB) {
        const uint64_t se = (ke - sb) < K2D_SUB - 1 ? ke : sb + K2D_SUB - 1;
        const uint32_t ns = (uint32_t)(se - sb) + 1;
        // the previous sub-chunk's readers are done with rk
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (uint32_t i = lane; i < ns; i += 64)
            rk[i] = 1.0 / (double)(sb + i);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll 1
        for (uint32_t g = 0; g < 8; ++g) {
            const uint32_t xl = 8 * g + xi;
            uint64_t m = 0, lo = 1, hi = 0;
            if (xl < nx) {
                m = q.x_m[g0 + xl];
                lo = q.x_klo[g0 + xl];
                hi = q.x_khi[g0 + xl];
                lo = lo > sb ? lo : sb;
                hi = hi < se ? hi : se;
            }
            const bool has = lo <= hi;
            const uint64_t glo = uniform_u64(wave_min_u64(has ? lo : ~0ull));
            const uint64_t ghi = uniform_u64(wave_max_u64(has ? hi : 0ull));
            uint64_t acc = 0;
            const double mf = (double)m;
            const uint32_t y1lo = (uint32_t)b.y1;
            for (uint64_t kk = glo; kk <= ghi; kk += 8 * K_UNROLL) {
                uint32_t off[K_UNROLL];
                bool act[K_UNROLL];
#pragma unroll
                for (int u = 0; u < K_UNROLL; ++u) {
                    const uint64_t k = kk + 8 * u + kj;
                    act[u] = k >= lo && k <= hi;
                    const double qd = mf * rk[act[u] ? (uint32_t)(k - sb) : 0u];
                    const double t = trunc(qd);
                    // t is floor(m/k) when qd < 2^32 and not near an integer
                    const bool fast = qd < 4294967296.0 && fabs(qd - t - 0.5) <= 0.5 - QEPS;
                    uint32_t ylo = (uint32_t)t;
                    if (act[u] && !fast)
                        ylo = (uint32_t)fix_quotient_any(m, k, t);
                    // y - y1 < 2^31: its low 32 bits are the difference of the low words
                    off[u] = act[u] ? ylo - y1lo : 0u;
                }
                acc += M_sum_masked32(b.words, off, act);
            }
            acc += __shfl_xor(acc, 1, 64);
            acc += __shfl_xor(acc, 2, 64);
            acc += __shfl_xor(acc, 4, 64);
            if (kj == g)
                mine += acc;
        }
    }
    const uint32_t xo = 8 * kj + xi;
    if (xo < nx)
        atomicAdd((unsigned long long *)&q.S[g0 + xo], (unsigned long long)mine);
}

// Explicit k part of one (tile, chunk) item: S[x] += M(floor(m_x / k)) for
// k in x's range [klo, khi] of this block.  Mode 0 tiles (k ranges of
// neighbouring x alike) use the 8 x 8 grid above over k-chunks; mode 1
// tiles use balanced runs of their pairs.
__device__ inline void k_item(const QueryArgs &q, const BlockArgs &b, uint32_t tile, uint64_t c,
                              double *rk, uint32_t wa, uint32_t wb)
{
    if (__builtin_amdgcn_readfirstlane(q.tile_mode[tile]) == 0) {
        k_item_2d(q, b, tile, c, rk, wa, wb);
        return;
    }
    // Balanced runs: the tile's pairs are numbered through an exclusive
    // prefix over its x; item c takes pairs [c K_BAL_PAIRS, ...) and splits
    // them into 64 equal contiguous runs, one per lane.  A lane walks its
    // run's k (one x at a time, K_UNROLL gathers in flight) and adds each x's
    // sum with one atomic.
    const uint32_t lane = lane_id();
    const uint32_t nx = __builtin_amdgcn_readfirstlane(q.tile_nx[tile]);
    const uint64_t g0 = uniform_u64(q.tile_g0[tile]);
    uint64_t m = 0, klo = 1, cnt = 0;
    if (lane < nx) {
        m = q.x_m[g0 + lane];
        klo = q.x_klo[g0 + lane];
        const uint64_t khi = q.x_khi[g0 + lane];
        cnt = klo <= khi ? khi - klo + 1 : 0;
    }
    uint64_t incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t t = __shfl_up(incl, o, 64);
        if (lane >= (uint32_t)o)
            incl += t;
    }
    const uint64_t T = readlane_u64(incl, 63);
    const uint64_t pa = c * K_BAL_PAIRS;
    const uint64_t pb = (T - pa) < K_BAL_PAIRS ? T : pa + K_BAL_PAIRS;
    uint64_t *sm = reinterpret_cast<uint64_t *>(rk);  // m, first k, prefix per x
    uint64_t *sk = sm + 64, *se = sm + 128;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    sm[lane] = m;
    sk[lane] = klo;
    se[lane] = incl - cnt;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint64_t p = pa + (pb - pa) * lane / 64;
    const uint64_t p1 = pa + (pb - pa) * (lane + 1) / 64;
    if (p >= p1)
        return;
    // x of pair p: the last x whose prefix is <= p (it has pairs left)
    uint32_t e = 0;
    for (uint32_t step = 32; step >= 1; step >>= 1)
        if (e + step < 64 && se[e + step] <= p)
            e += step;
    while (p < p1) {
        const uint64_t me = sm[e];
        const uint64_t pend = e < 63 ? se[e + 1] : T;  // first pair of the next x
        const uint64_t stop = pend < p1 ? pend : p1;
        const uint64_t kend = sk[e] + (stop - se[e]);  // exclusive
        const double mf = (double)me;
        uint64_t acc = 0;
        for (uint64_t k = sk[e] + (p - se[e]); k < kend; k += K_UNROLL) {
            uint64_t off[K_UNROLL];
            bool act[K_UNROLL];
#pragma unroll
            for (int u = 0; u < K_UNROLL; ++u) {
                const uint64_t kk = k + u;
                act[u] = kk < kend;
                off[u] = 0;
                if (act[u])
                    off[u] = fix_quotient_any(me, kk, trunc(mf / (double)kk)) - b.y1;
            }
            acc += M_sum_masked(b.words, off, act);
        }
        atomicAdd((unsigned long long *)&q.S[g0 + e], (unsigned long long)acc);
        p = stop;
        while (p < p1 && e < 63 && se[e + 1] <= p)  // next x with pairs
            ++e;
    }
}

// Persistent update kernel of one block: wave w starts on item w and then
// takes further items from a device counter until the block's items are
// exhausted (a block with fewer items than waves costs no atomics beyond
// one per item).  Three workgroups per CU (12 waves, up to 168 VGPRs): the
// run-length passes keep 16 x of quotient state per lane, which at four
// workgroups (128 VGPRs) spilled to scratch.
__global__ __launch_bounds__(UPD_THREADS, 3) void k_update(QueryArgs q, BlockArgs b_in, uint32_t wa,
                                                           uint32_t wb)
{
    // per wave: compacted run-length entries or explicit-k reciprocals
    static_assert(RL_ENT_CAP * 2 >= K2D_SUB * 8, "LDS slice too small");
    static_assert(RL_ENT_CAP / 4 >= K2D_SUB + 8 * K2F_UNROLL, "fast walk reads past the slice");
    __shared__ double wave_lds[UPD_THREADS / 64][RL_ENT_CAP / 4];
    const BlockArgs b = load_block(b_in);
    const uint32_t lane = lane_id();
    double *wl = wave_lds[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)];
    uint16_t *ent = reinterpret_cast<uint16_t *>(wl);
    const uint64_t total = uniform_u64(q.tile_items[q.ntiles]);
    const uint32_t nwaves = gridDim.x * (UPD_THREADS / 64);
    uint64_t item = __builtin_amdgcn_readfirstlane(blockIdx.x * (UPD_THREADS / 64) +
                                                   (threadIdx.x >> 6));
    for (;;) {
        if (item >= total)
            break;
        const uint32_t tile =
            __builtin_amdgcn_readfirstlane(find_tile(q.tile_items, q.ntiles, item));
        const uint64_t local = uniform_u64(item - q.tile_items[tile]);
        const uint32_t nmu = __builtin_amdgcn_readfirstlane(q.tile_nmu[tile]);
        if (local < nmu)
            mu_item(q, b, tile, local, ent);
        else
            k_item(q, b, tile, local - nmu, wl, wa, wb);
        // One ticket per wave.  Every lane executes the atomic (lane 0 adds
        // 1, the others 0) so no divergent branch guards it, and readfirstlane
        // turns the ticket into a scalar: the exit test is a uniform branch,
        // and the compiler cannot split the wave across loop iterations
        // around the cross-lane operations in the body.
        const uint32_t it = atomicAdd(q.counter, lane == 0 ? 1u : 0u);
        item = (uint64_t)nwaves + (uint32_t)__builtin_amdgcn_readfirstlane(it);
    }
}

hipError_t launch_update(const QueryArgs &q, const BlockArgs &b, uint32_t grid, hipStream_t s,
                         uint32_t wa, uint32_t wb)
{
    hipLaunchKernelGGL(k_update, dim3(grid), dim3(UPD_THREADS), 0, s, q, b, wa, wb);
    return hipGetLastError();
}

// Explicit-k pairs of the band [2^wa, 2^wb), y-major: one workgroup per
// (group of EKW_TILES tiles, run of EKW_RUN consecutive windows of EKW_Y y),
// the groups of one run consecutive in dispatch order (they share its
// records in L2).  Each window's records are staged in LDS with coalesced
// loads in turn (a window with no pair of the group is skipped); each
// wave takes one tile and, for its x, the k whose quotient lies in the
// window, k in [floor(m / (Y0 + EKW_Y)) + 1, floor(m / Y0)] (within the
// block's k range), one lane per x with a reciprocal per pair and the
// records read from LDS; the lane's sum over the run leaves with one atomic.
// Offsets are taken from Y0 (the window is no longer than Y0,
// so the fused quotient rule above holds with y1 = Y0).  Windows start at
// ystart (a multiple of EKW_Y, at least EKW_Y) and cover [ystart, yend);
// yend <= 2^31.
constexpr uint32_t EKW_Y = 1u << EKW_SHIFT;
constexpr uint32_t EKW_REC = EKW_Y / 32;  // 4096 records = 64 KiB
constexpr uint32_t EKW_NONE = EKW_REC * 32;  // offset of the empty record after them
constexpr int EKW_THREADS = 1024;
constexpr uint32_t EKW_TILES = EKW_THREADS / 64;
constexpr int EKW_UNROLL = 4;  // LDS reads per lane and batch (eight spill at 64 VGPRs)
constexpr uint32_t EKW_RUN = 8;  // consecutive windows per workgroup

// floor(a / d) for a < 2^32, 1 <= d < 2^32: an fp64 estimate (within one
// of the quotient) and one integer correction.
__device__ inline uint32_t div_small(uint32_t a, uint32_t d)
{
    uint32_t qv = (uint32_t)((double)a * rcp_1ulp((double)d));
    const int64_t r = (int64_t)a - (int64_t)qv * (int64_t)d;
    if (r < 0)
        qv -= 1;
    else if (r >= (int64_t)d)
        qv += 1;
    return qv;
}

__global__ __launch_bounds__(EKW_THREADS, 8) void k_ek_window(QueryArgs q, BlockArgs b_in,
                                                           uint64_t ystart, uint64_t yend)
{
    __shared__ u32x4 win[EKW_REC + 1];
    // per wave: its largest count of pairs in the window, in two sets used
    // by alternate windows (a wave may write the next window's flag while
    // another still reads this one's; reusing a set needs the next barrier,
    // which every wave reaches only after its reads)
    __shared__ uint32_t wave_busy[2][EKW_TILES];
    const BlockArgs b = load_block(b_in);
    const uint32_t tid = threadIdx.x, lane = lane_id();
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // this wave's tile; lane l holds its x l (an empty k range past the tile)
    const uint32_t tile = blockIdx.x * EKW_TILES + wave;
    uint32_t nx = 0;
    uint64_t g0 = 0, m_l = 0, klo_l = 1, khi_l = 0;
    bool act = false;
    if (tile < q.ntiles) {
        nx = __builtin_amdgcn_readfirstlane(q.tile_nx[tile]);
        g0 = uniform_u64(q.tile_g0[tile]);
        if (lane < nx) {
            m_l = q.x_m[g0 + lane];
            klo_l = q.x_klo[g0 + lane];
            khi_l = q.x_khi[g0 + lane];
        }
        act = band_tile(q, b, uniform_u64(wave_max_u64(m_l)), q.tile_mode[tile]);
    }
    const uint32_t mh = act ? (uint32_t)(m_l >> EKW_SHIFT) : 0u;  // m < 2^48: < 2^31
    const double mf = (double)m_l;
    const RecLds src{win};
    const uint32_t rec_bytes = ((uint32_t)((b.y2 - b.y1) >> 5) + 1u) * 16u;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(b.words, (short)0, (int)rec_bytes, 0x00020000);
    if (tid == 0)
        win[EKW_REC] = u32x4{0u, 0u, 0u, 0u};
    uint32_t dp = 0, dn = 0;  // the lane's x, over every window of the run
    uint64_t ms = 0;
    for (uint32_t r = 0; r < EKW_RUN; ++r) {
        const uint64_t Y0 = ystart + ((uint64_t)blockIdx.y * EKW_RUN + r) * EKW_Y;
        if (Y0 >= yend || Y0 > b.y2)  // the same for the whole workgroup
            break;
        // the window's k: floor(m / (a 2^17)) = floor(floor(m / 2^17) / a)
        uint64_t lo = 1, hi = 0;
        if (act) {
            const uint32_t a = (uint32_t)(Y0 >> EKW_SHIFT);  // < 2^14 (Y0 < 2^31)
            const uint64_t kw_hi = div_small(mh, a), kw_lo = (uint64_t)div_small(mh, a + 1) + 1;
            lo = klo_l > kw_lo ? klo_l : kw_lo;
            hi = khi_l < kw_hi ? khi_l : kw_hi;
        }
        const uint32_t cnt = lo <= hi ? (uint32_t)(hi - lo) + 1u : 0u;  // k < 2^31
        const uint32_t cmax = (uint32_t)uniform_u64(wave_max_u64(cnt));
        if (lane == 0)
            wave_busy[r & 1u][wave] = cmax;
        __syncthreads();  // the previous window's readers are done; flags written
        uint32_t any = 0;
#pragma unroll
        for (uint32_t w = 0; w < EKW_TILES; ++w)
            any |= wave_busy[r & 1u][w];
        if (any == 0)  // no pair of the group in this window: skip its records
            continue;
        const uint32_t base = (uint32_t)((Y0 - b.y1) >> 5) * 16u;  // < 2^27
        for (uint32_t i = tid; i < EKW_REC; i += EKW_THREADS)
            win[i] = __builtin_amdgcn_raw_buffer_load_b128(rs, base + i * 16u, 0, 0);
        __syncthreads();
        // lane l walks the k of its x in this window (m 2^17 / Y0^2 of
        // them: a few to thousands), reciprocals per pair
        const double ny0 = -(double)Y0;
        double kd = (double)lo;  // k of the batch's first pair (exact: k < 2^32)
        for (uint32_t j = 0; j < cmax; j += EKW_UNROLL, kd += (double)EKW_UNROLL) {
            K2Batch<EKW_UNROLL> t;
#pragma unroll
            for (int u = 0; u < EKW_UNROLL; ++u) {
                const uint32_t o = (uint32_t)fma(mf, rcp_up(kd + (double)u), ny0);
                t.off[u] = j + (uint32_t)u < cnt ? o : EKW_NONE;
            }
#pragma unroll
            for (int u = 0; u < EKW_UNROLL; ++u)
                t.rec[u] = src(t.off[u]);
            k2_consume<EKW_UNROLL>(t, dp, dn, ms);
        }
    }
    const uint64_t mine = ms + (uint64_t)(int64_t)(int32_t)(dp - dn);
    if (act && lane < nx && mine)
        atomicAdd((unsigned long long *)&q.S[g0 + lane], (unsigned long long)mine);
}

hipError_t launch_ek_window(const QueryArgs &q, const BlockArgs &b, uint64_t ystart,
                            uint64_t yend, hipStream_t s)
{
    // grid: tile groups along x, windows along y (each dimension's count of
    // work-items must stay below 2^32; a one-dimensional grid of both would
    // pass it for large batches)
    const uint32_t ngroups = (q.ntiles + EKW_TILES - 1) / EKW_TILES;
    const uint32_t nwin = (uint32_t)((yend - ystart + EKW_Y - 1) / EKW_Y);
    const uint32_t nruns = (nwin + EKW_RUN - 1) / EKW_RUN;
    if ((uint64_t)ngroups * EKW_THREADS >= (1ull << 32) || nruns >= (1u << 16))
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_ek_window, dim3(ngroups, nruns), dim3(EKW_THREADS), 0, s, q, b, ystart,
                       yend);
    return hipGetLastError();
}

// ====================================================================
// a4: finalize.  A[x] = 1 - S[x] - sum_{k=2}^{floor(L/x)} A[kx], for x from
// L down to 1 (Section 2), one workgroup per query.  The x are taken in
// dyadic levels (floor(h/2), h]: every dependency kx >= 2x > h lies in an
// earlier level, so a level's x are independent and there are only
// ceil(log2 L) + 1 barriers.
// ====================================================================
constexpr int FIN_THREADS = 1024;

// Entry of (x, m) in the keyed group starting at entry g0 with key_off base
// kb (x <= L, and (x, m) is one of the group's pairs): binary search among
// the sorted m of x's entries.
__device__ inline uint64_t key_find(const QueryArgs &q, uint64_t g0, uint64_t kb, uint64_t x,
                                    uint64_t m)
{
    uint64_t lo = g0 + q.key_off[kb + x - 1];
    uint64_t hi = g0 + q.key_off[kb + x];
    while (hi - lo > 1) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (q.x_m[mid] <= m)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Finalize of a keyed group: the same recursion over entries, with A[kx]
// taken from the entry (kx, floor(m/k)), since floor(floor(n/x)/k) =
// floor(n/(kx)).  Levels of x as in k_finalize; a level's entries are
// independent.
__device__ void finalize_keyed(const QueryArgs &q, uint32_t qi, uint64_t *red)
{
    const uint64_t L = q.q_L[qi];
    const uint64_t g0 = q.q_g0[qi];
    const uint64_t kb = q.q_koff[qi];
    uint64_t *A = reinterpret_cast<uint64_t *>(q.A);
    const uint32_t tid = threadIdx.x, lane = lane_id();
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (uint64_t hi = L, lo = L / 2; hi >= 1; hi = lo, lo = lo / 2) {
        const uint64_t e0 = g0 + q.key_off[kb + lo], e1 = g0 + q.key_off[kb + hi];
        const uint64_t ne = e1 - e0;
        if (ne >= FIN_THREADS) {
            for (uint64_t e = e0 + tid; e < e1; e += FIN_THREADS) {
                const uint64_t x = q.key_x[e], m = q.x_m[e];
                uint64_t s = 1 - q.S[e];
                const uint64_t j = L / x;
                for (uint64_t k = 2; k <= j; ++k)
                    s -= A[key_find(q, g0, kb, k * x, m / k)];
                A[e] = s;
            }
        } else if (ne > 4) {
            uint32_t gsz = 1;
            while (gsz < 64 && (uint64_t)gsz * 2 * ne <= FIN_THREADS)
                gsz *= 2;
            const uint32_t ngroups = FIN_THREADS / gsz;
            const uint32_t grp = tid / gsz, sub = tid % gsz;
            for (uint64_t base = 0; base < ne; base += ngroups) {  // same trip count for all
                const uint64_t ei = base + grp;
                const bool active = ei < ne;
                const uint64_t e = e0 + ei;
                uint64_t s = 0;
                uint64_t x = 1, m = 0;
                if (active) {
                    x = q.key_x[e];
                    m = q.x_m[e];
                    const uint64_t j = L / x;
                    for (uint64_t k = 2 + sub; k <= j; k += gsz)
                        s += A[key_find(q, g0, kb, k * x, m / k)];
                }
                for (uint32_t o = gsz / 2; o >= 1; o >>= 1)
                    s += __shfl_xor(s, (int)o, 64);
                if (active && sub == 0)
                    A[e] = 1 - q.S[e] - s;
            }
        } else {
            for (uint64_t e = e0; e < e1; ++e) {
                const uint64_t x = q.key_x[e], m = q.x_m[e];
                const uint64_t j = L / x;
                uint64_t s = 0;
                for (uint64_t k = 2 + tid; k <= j; k += FIN_THREADS)
                    s += A[key_find(q, g0, kb, k * x, m / k)];
                s = wave_sum_u64(s);
                if (lane == 0)
                    red[wave] = s;
                __syncthreads();
                if (tid == 0) {
                    uint64_t t = 0;
                    for (int w = 0; w < FIN_THREADS / 64; ++w)
                        t += red[w];
                    A[e] = 1 - q.S[e] - t;
                }
                __syncthreads();
            }
        }
        __syncthreads();
    }
}

// One level (lo, hi] of a keyed group's finalize across the whole grid (the
// group of a dense window can hold 10^7 entries, far too many for one
// workgroup): gsz lanes (a power of two up to 64, within one wave) share
// one entry, its terms k strided over them.
__global__ __launch_bounds__(256) void k_finalize_keyed_level(QueryArgs q, uint32_t qi, uint64_t lo,
                                                             uint64_t hi, uint32_t gsz)
{
    const uint64_t L = q.q_L[qi], g0 = q.q_g0[qi], kb = q.q_koff[qi];
    uint64_t *A = reinterpret_cast<uint64_t *>(q.A);
    const uint64_t e0 = g0 + q.key_off[kb + lo], e1 = g0 + q.key_off[kb + hi];
    const uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t ei = gt / gsz;
    const uint32_t sub = (uint32_t)(gt % gsz);
    const bool active = ei < e1 - e0;
    const uint64_t e = e0 + ei;
    uint64_t s = 0;
    if (active) {
        const uint64_t x = q.key_x[e], m = q.x_m[e];
        const uint64_t j = L / x;
        for (uint64_t k = 2 + sub; k <= j; k += gsz)
            s += A[key_find(q, g0, kb, k * x, m / k)];
    }
    for (uint32_t o = gsz / 2; o >= 1; o >>= 1)
        s += __shfl_xor(s, (int)o, 64);
    if (active && sub == 0)
        A[e] = 1 - q.S[e] - s;
}

hipError_t launch_finalize_keyed_level(const QueryArgs &q, uint32_t qi, uint64_t lo, uint64_t hi,
                                       uint64_t entries, uint32_t gsz, hipStream_t s)
{
    const uint64_t threads = entries * gsz;
    hipLaunchKernelGGL(k_finalize_keyed_level, dim3((uint32_t)((threads + 255) / 256)), dim3(256),
                       0, s, q, qi, lo, hi, gsz);
    return hipGetLastError();
}

__global__ __launch_bounds__(FIN_THREADS) void k_finalize(QueryArgs q, const uint32_t *qlist)
{
    __shared__ uint64_t red[FIN_THREADS / 64];
    const uint32_t qi = qlist ? qlist[blockIdx.x] : blockIdx.x;
    if (q.q_koff[qi] != ~0ull) {
        finalize_keyed(q, qi, red);
        return;
    }
    const uint64_t L = q.q_L[qi];
    const uint64_t g0 = q.q_g0[qi];
    const uint64_t *S = q.S + g0;
    uint64_t *A = reinterpret_cast<uint64_t *>(q.A + g0);  // A[x-1], wrapping arithmetic
    const uint32_t tid = threadIdx.x, lane = lane_id();
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (uint64_t hi = L, lo = L / 2; hi >= 1; hi = lo, lo = lo / 2) {
        const uint64_t nx = hi - lo;  // x in (lo, hi]
        if (nx >= FIN_THREADS) {
            for (uint64_t x = lo + 1 + tid; x <= hi; x += FIN_THREADS) {
                uint64_t s = 1 - S[x - 1];
                const uint64_t j = L / x;
                for (uint64_t k = 2; k <= j; ++k)
                    s -= A[k * x - 1];
                A[x - 1] = s;
            }
        } else if (nx > 4) {
            // groups of gsz lanes (a power of two <= 64) share one x
            uint32_t gsz = 1;
            while (gsz < 64 && (uint64_t)gsz * 2 * nx <= FIN_THREADS)
                gsz *= 2;
            const uint32_t ngroups = FIN_THREADS / gsz;
            const uint32_t grp = tid / gsz, sub = tid % gsz;
            for (uint64_t base = 0; base < nx; base += ngroups) {  // same trip count for all
                const uint64_t xi = base + grp;
                const bool active = xi < nx;
                const uint64_t x = lo + 1 + xi;
                uint64_t s = 0;
                if (active) {
                    const uint64_t j = L / x;
                    for (uint64_t k = 2 + sub; k <= j; k += gsz)
                        s += A[k * x - 1];
                }
                for (uint32_t o = gsz / 2; o >= 1; o >>= 1)
                    s += __shfl_xor(s, (int)o, 64);
                if (active && sub == 0)
                    A[x - 1] = 1 - S[x - 1] - s;
            }
        } else {
            // a handful of x with many terms each: the whole workgroup per x
            for (uint64_t x = lo + 1; x <= hi; ++x) {
                const uint64_t j = L / x;
                uint64_t s = 0;
                for (uint64_t k = 2 + tid; k <= j; k += FIN_THREADS)
                    s += A[k * x - 1];
                s = wave_sum_u64(s);
                if (lane == 0)
                    red[wave] = s;
                __syncthreads();
                if (tid == 0) {
                    uint64_t t = 0;
                    for (int w = 0; w < FIN_THREADS / 64; ++w)
                        t += red[w];
                    A[x - 1] = 1 - S[x - 1] - t;
                }
                __syncthreads();
            }
        }
        __syncthreads();
    }
}

hipError_t launch_finalize(const QueryArgs &q, const uint32_t *qlist, uint32_t count,
                           hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(count), dim3(FIN_THREADS), 0, s, q, qlist);
    return hipGetLastError();
}

__global__ void k_collect(QueryArgs q, int64_t *out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= q.nq)
        return;
    const uint64_t kb = q.q_koff[i];
    out[i] = kb == ~0ull ? q.A[q.q_g0[i]] : q.A[key_find(q, q.q_g0[i], kb, 1, q.q_n[i])];
}

__global__ void k_keyed_byproducts(QueryArgs q, uint32_t qi, uint64_t count, int64_t *out)
{
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (c > count)
        return;
    out[c - 1] = q.A[key_find(q, q.q_g0[qi], q.q_koff[qi], c, q.q_n[qi] / c)];
}

hipError_t launch_keyed_byproducts(const QueryArgs &q, uint32_t qi, uint64_t count, int64_t *out,
                                   hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_keyed_byproducts, dim3((uint32_t)((count + 255) / 256)), dim3(256), 0, s,
                       q, qi, count, out);
    return hipGetLastError();
}

hipError_t launch_collect(const QueryArgs &q, int64_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_collect, dim3((q.nq + 255) / 256), dim3(256), 0, s, q, out);
    return hipGetLastError();
}

// ====================================================================
// Interval sweep (Section 6): every M(n) on [a, b] from an exact M(a) and
// the sieve records of the blocks covering [a, b], and the n where
// M(n)/sqrt(n) is smallest and largest.  The blocks are sieved with the
// carry starting at 0, so a record holds M(y) - M(start - 1); *off turns
// that into M(y).
// ====================================================================

// |m|^2 n as a 192-bit integer (|m| < 2^63, n < 2^64), low word first.
struct U192 {
    uint64_t w0, w1, w2;
};

__device__ inline U192 sq_times(uint64_t a, uint64_t n)
{
    const uint64_t l = a * a, h = __umul64hi(a, a);  // a^2 = h 2^64 + l
    U192 r;
    r.w0 = l * n;
    const uint64_t t = __umul64hi(l, n);
    r.w1 = t + h * n;
    r.w2 = __umul64hi(h, n) + (r.w1 < t ? 1u : 0u);
    return r;
}

__device__ inline int cmp192(const U192 &x, const U192 &y)
{
    if (x.w2 != y.w2)
        return x.w2 < y.w2 ? -1 : 1;
    if (x.w1 != y.w1)
        return x.w1 < y.w1 ? -1 : 1;
    if (x.w0 != y.w0)
        return x.w0 < y.w0 ? -1 : 1;
    return 0;
}

// Sign of m1 / sqrt(n1) - m2 / sqrt(n2) (n1, n2 >= 1), without rounding:
// signs first, then m1^2 n2 against m2^2 n1 (reversed for negative m).
__device__ inline int ratio_cmp(int64_t m1, uint64_t n1, int64_t m2, uint64_t n2)
{
    const int s1 = (m1 > 0) - (m1 < 0), s2 = (m2 > 0) - (m2 < 0);
    if (s1 != s2)
        return s1 < s2 ? -1 : 1;
    if (s1 == 0)
        return 0;
    const uint64_t a1 = m1 < 0 ? 0 - (uint64_t)m1 : (uint64_t)m1;
    const uint64_t a2 = m2 < 0 ? 0 - (uint64_t)m2 : (uint64_t)m2;
    int c;
    if ((a1 | a2) >> 32 == 0) {  // squares fit 64 bits: 128-bit products
        const uint64_t q1 = a1 * a1, q2 = a2 * a2;
        const uint64_t h1 = __umul64hi(q1, n2), h2 = __umul64hi(q2, n1);
        const uint64_t l1 = q1 * n2, l2 = q2 * n1;
        c = h1 != h2 ? (h1 < h2 ? -1 : 1) : (l1 != l2 ? (l1 < l2 ? -1 : 1) : 0);
    } else {
        c = cmp192(sq_times(a1, n2), sq_times(a2, n1));
    }
    return s1 > 0 ? c : -c;
}

// Candidate (n1, m1) beats (n2, m2) for the minimum (dir = 1) or the
// maximum (dir = -1) of m / sqrt(n); n = 0 is "none"; equal ratios keep the
// smaller n.  A total order, so any reduction order gives the same winner.
__device__ inline bool beats(uint64_t n1, int64_t m1, uint64_t n2, int64_t m2, int dir)
{
    if (n1 == 0)
        return false;
    if (n2 == 0)
        return true;
    const int c = ratio_cmp(m1, n1, m2, n2) * dir;
    return c < 0 || (c == 0 && n1 < n2);
}

struct Extremes {
    uint64_t nmin, nmax;
    int64_t mmin, mmax;
};

__device__ inline void merge_extremes(Extremes &e, const Extremes &o)
{
    if (beats(o.nmin, o.mmin, e.nmin, e.mmin, 1)) {
        e.nmin = o.nmin;
        e.mmin = o.mmin;
    }
    if (beats(o.nmax, o.mmax, e.nmax, e.mmax, -1)) {
        e.nmax = o.nmax;
        e.mmax = o.mmax;
    }
}

__device__ inline Extremes wave_extremes(Extremes e)
{
    for (int o = 32; o >= 1; o >>= 1) {
        Extremes t;
        t.nmin = __shfl_xor(e.nmin, o, 64);
        t.mmin = __shfl_xor(e.mmin, o, 64);
        t.nmax = __shfl_xor(e.nmax, o, 64);
        t.mmax = __shfl_xor(e.mmax, o, 64);
        merge_extremes(e, t);
    }
    return e;
}

// Workgroup reduction of e (every thread passes its own); the result is
// valid in thread 0.
__device__ inline Extremes wg_extremes(Extremes e, Extremes *lds)
{
    e = wave_extremes(e);
    const uint32_t wave = threadIdx.x >> 6;
    if (lane_id() == 0)
        lds[wave] = e;
    __syncthreads();
    if (threadIdx.x == 0)
        for (uint32_t k = 1; k < blockDim.x / 64; ++k)
            merge_extremes(e, lds[k]);
    return e;
}

__global__ void k_interval_base(BlockArgs b_in, uint64_t a, int64_t m_a, int64_t *off)
{
    const BlockArgs b = load_block(b_in);
    if (threadIdx.x == 0)
        *off = m_a - M_at(b.words, a - b.y1);
}

hipError_t launch_interval_base(const BlockArgs &b, uint64_t a, int64_t m_a, int64_t *off,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_interval_base, dim3(1), dim3(64), 0, s, b, a, m_a, off);
    return hipGetLastError();
}

// One thread per 32-y record (grid-stride, so a thread meets its y in
// increasing order, each after its current candidates): M(y) is the
// record's value plus the running +-1 bits.  As a later y with an equal
// ratio loses, a record can only hold a new minimum if the ratio bound
// mlo / sqrt(y) (M at least the value before it minus its -1 count, y at the
// end that makes the bound smallest) is strictly below the current one, and
// likewise for the maximum; other records are skipped after that exact test.
__global__ __launch_bounds__(IV_THREADS) void k_interval_extreme(BlockArgs b_in, uint64_t lo,
                                                                 uint64_t hi, const int64_t *off,
                                                                 uint64_t *part)
{
    const BlockArgs b = load_block(b_in);
    __shared__ Extremes lds[IV_THREADS / 64];
    const int64_t base = *off;
    const uint64_t r0 = (lo - b.y1) >> 5, r1 = (hi - b.y1) >> 5;
    Extremes e = {0, 0, 0, 0};
    for (uint64_t r = r0 + (uint64_t)blockIdx.x * IV_THREADS + threadIdx.x; r <= r1;
         r += (uint64_t)gridDim.x * IV_THREADS) {
        const ulonglong2 rec = *reinterpret_cast<const ulonglong2 *>(b.words + 2 * r);
        const uint32_t pos = (uint32_t)rec.x, neg = (uint32_t)(rec.x >> 32);
        const uint64_t y0 = b.y1 + 32 * r;
        const uint32_t jlo = y0 < lo ? (uint32_t)(lo - y0) : 0u;
        const uint32_t jhi = hi - y0 < 31 ? (uint32_t)(hi - y0) : 31u;
        const int64_t m0 = (int64_t)rec.y + base;
        const int64_t mlo = m0 - __popc(neg), mhi = m0 + __popc(pos);
        const uint64_t ylo = y0 + jlo, yhi = y0 + jhi;
        const bool pmin = e.nmin == 0 || ratio_cmp(mlo, mlo < 0 ? ylo : yhi, e.mmin, e.nmin) < 0;
        const bool pmax = e.nmax == 0 || ratio_cmp(mhi, mhi < 0 ? yhi : ylo, e.mmax, e.nmax) > 0;
        if (!pmin && !pmax)
            continue;
        int64_t m = m0;
        for (uint32_t j = 0; j <= jhi; ++j) {
            m += (int64_t)((pos >> j) & 1u) - (int64_t)((neg >> j) & 1u);
            if (j < jlo)
                continue;
            const uint64_t y = y0 + j;
            // below a negative minimum / above a positive maximum only
            if (pmin && (e.mmin >= 0 || m < e.mmin) && beats(y, m, e.nmin, e.mmin, 1)) {
                e.nmin = y;
                e.mmin = m;
            }
            if (pmax && (e.mmax <= 0 || m > e.mmax) && beats(y, m, e.nmax, e.mmax, -1)) {
                e.nmax = y;
                e.mmax = m;
            }
        }
    }
    e = wg_extremes(e, lds);
    if (threadIdx.x == 0) {
        uint64_t *pw = part + 4 * (size_t)blockIdx.x;
        const Extremes prev = {pw[0], pw[2], (int64_t)pw[1], (int64_t)pw[3]};
        merge_extremes(e, prev);
        pw[0] = e.nmin;
        pw[1] = (uint64_t)e.mmin;
        pw[2] = e.nmax;
        pw[3] = (uint64_t)e.mmax;
    }
}

hipError_t launch_interval_extreme(const BlockArgs &b, uint64_t lo, uint64_t hi,
                                   const int64_t *off, uint64_t *part, hipStream_t s)
{
    hipLaunchKernelGGL(k_interval_extreme, dim3(IV_WGS), dim3(IV_THREADS), 0, s, b, lo, hi, off,
                       part);
    return hipGetLastError();
}

__global__ void k_interval_values(BlockArgs b_in, uint64_t lo, uint64_t count, const int64_t *off,
                                  int64_t *dst)
{
    const BlockArgs b = load_block(b_in);
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        dst[i] = M_at(b.words, lo + i - b.y1) + *off;
}

hipError_t launch_interval_values(const BlockArgs &b, uint64_t lo, uint64_t count,
                                  const int64_t *off, int64_t *dst, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_interval_values, dim3((uint32_t)((count + 255) / 256)), dim3(256), 0, s,
                       b, lo, count, off, dst);
    return hipGetLastError();
}

__global__ __launch_bounds__(IV_THREADS) void k_interval_final(BlockArgs b_in,
                                                               const uint64_t *part,
                                                               uint64_t n_end, const int64_t *off,
                                                               int64_t *res)
{
    const BlockArgs b = load_block(b_in);
    __shared__ Extremes lds[IV_THREADS / 64];
    Extremes e = {0, 0, 0, 0};
    for (uint32_t w = threadIdx.x; w < IV_WGS; w += IV_THREADS) {
        const uint64_t *pw = part + 4 * (size_t)w;
        const Extremes o = {pw[0], pw[2], (int64_t)pw[1], (int64_t)pw[3]};
        merge_extremes(e, o);
    }
    e = wg_extremes(e, lds);
    if (threadIdx.x == 0) {
        res[0] = (int64_t)e.nmin;
        res[1] = e.mmin;
        res[2] = (int64_t)e.nmax;
        res[3] = e.mmax;
        res[4] = M_at(b.words, n_end - b.y1) + *off;
    }
}

hipError_t launch_interval_final(const BlockArgs &b, const uint64_t *part, uint64_t n_end,
                                 const int64_t *off, int64_t *res, hipStream_t s)
{
    hipLaunchKernelGGL(k_interval_final, dim3(1), dim3(IV_THREADS), 0, s, b, part, n_end, off,
                       res);
    return hipGetLastError();
}

// ====================================================================
// diagnostics
// ====================================================================
__global__ void k_debug_div(const uint64_t *n, const uint64_t *d, uint64_t *qo, size_t count)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count)
        return;
    uint64_t mul;
    uint32_t sh1, sh2;
    gm_magic((uint32_t)d[i], mul, sh1, sh2);
    qo[i] = gm_div(n[i], mul, sh1, sh2);
}

hipError_t launch_debug_div(const uint64_t *n, const uint64_t *d, uint64_t *q, size_t count,
                            hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_debug_div, dim3((uint32_t)((count + 255) / 256)), dim3(256), 0, s, n, d,
                       q, count);
    return hipGetLastError();
}

// mu(y) and M(y) (relative to the block's carry) for y in [y_first, y_first+count)
__global__ void k_debug_mu(BlockArgs b_in, uint64_t y_first, uint32_t count, int8_t *mu, int64_t *mert)
{
    const BlockArgs b = load_block(b_in);
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count)
        return;
    const uint64_t off = y_first + i - b.y1;
    const uint64_t w = off >> 6;
    const uint32_t bt = (uint32_t)(off & 63);
    uint64_t nz, ng;
    word_masks(b.words, w, nz, ng);
    mu[i] = ((nz >> bt) & 1) ? (((ng >> bt) & 1) ? -1 : 1) : 0;
    if (mert)
        mert[i] = M_at(b.words, off);
}

hipError_t launch_debug_mu(const BlockArgs &b, uint64_t y_first, uint32_t count, int8_t *mu,
                           int64_t *mert, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_debug_mu, dim3((count + 255) / 256), dim3(256), 0, s, b, y_first, count,
                       mu, mert);
    return hipGetLastError();
}

}  // namespace mrt
