// Internal declarations shared by the kernel file and the host runtime of
// the gfx950 Mertens library.  Not part of the public ABI (include/mertens.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrt {

// ---------------------------------------------------------------- constants
// Sieve segment: one byte per y in LDS (128 KB), processed by one workgroup.
constexpr uint32_t SEG = 1u << 17;
constexpr uint32_t SEG_WORDS = SEG / 64;     // 64-y mask words per segment
constexpr int SIEVE_THREADS = 1024;          // 16 waves, 2 mask words per thread
// Pre-sieved pattern: log sums of 2,3,5,7,11,13 and square flags of 4 and 9
// repeat with period lcm(2,3,5,7,11,13,4,9) = 180180.  It is stored in the
// sieve's LDS layout (32-y groups, y offset t of a group in word t & 7,
// byte t >> 3) in eight copies that start 0, 4, ..., 28 pattern bytes late,
// so every segment (which starts at a multiple of 4 in the pattern) is one
// run of whole 32-byte groups of one copy.
constexpr uint32_t PAT = 180180;
constexpr uint32_t PAT_COPIES = 8;
constexpr uint32_t PAT_WORDS = ((PAT + SEG + 31) / 32) * 8;  // uint32 per copy
// Sieving primes below this bound (>= 64 multiples per segment) are walked by
// a whole wavefront, lane i taking the i-th multiple; larger ones by one lane.
constexpr uint32_t SMALL_P = SEG / 64;
// Squares of primes up to this bound are flagged in LDS by whole wavefronts;
// a larger square (> 2^20 > SEG) meets a segment at most once: per block,
// one thread per prime lists its multiples in per-segment buckets of
// SQ_BUCKET entries (a segment whose bucket overflows scans every prime).
constexpr uint32_t SQ_LDS_P = 1024;
constexpr uint32_t SQ_BUCKET = 64;
// Primes above SEG meet a segment at most once; when a block has many of
// them, BK_WGS workgroups (each a fixed share of those primes) list their
// multiples into per-segment buckets in two passes (count, fill), so the
// sieve reads its hits instead of testing every such prime.
#ifndef MERTENS_BK_WGS
#define MERTENS_BK_WGS 512
#endif
constexpr uint32_t BK_WGS = MERTENS_BK_WGS, BK_THREADS = 1024;
constexpr uint32_t MAX_SEGS = (1u << 31) / SEG;  // segments of the longest block
// The fill pass lists hits per group of BK_GROUP_SEGS segments (2^24 y)
// first, and a second pass spreads each group over its segments: both
// write into few runs at a time, which the L2 turns into whole-line writes.
constexpr uint32_t BK_GROUP_SEGS = 128, BK_GROUP_SHIFT = 24;
static_assert(BK_GROUP_SEGS * SEG == (1u << BK_GROUP_SHIFT), "group size");
static_assert(MAX_SEGS / BK_GROUP_SEGS <= MAX_SEGS, "group counters fit the LDS array");
// Interval sweep: workgroups of the extreme reduction (each keeps its own
// running candidates across the blocks of one interval).
constexpr uint32_t IV_WGS = 2048, IV_THREADS = 256;
// First index of the prime table that is sieved (table starts at 5; the
// pattern covers 5, 7, 11, 13, so sieving starts at 17 = index 4).
constexpr uint32_t FIRST_SIEVED = 4;
// Windows of the y-major explicit-k pass (k_ek_window): 2^EKW_SHIFT y, whose
// 16-byte records fill 64 KiB of LDS.
constexpr uint32_t EKW_SHIFT = 17;
constexpr int TILE = 64;                     // x per tile = one wavefront
// explicit-k pairs per balanced work item (tiles whose x have k ranges too
// different for the 8 x 8 walk): 256 per lane
constexpr uint64_t K_BAL_PAIRS = 64 * 256;
constexpr int UPD_THREADS = 256;             // 4 independent waves per workgroup

// ---------------------------------------------------------------- arguments
// The per-block values of a y-block [y1, y2] (y1 a multiple of SEG).  The
// kernels read them from device memory (BlockArgs::bp) so that one captured
// graph of the block pipeline can be replayed for every block.
struct BlockParams {
    uint64_t y1, y2;
    uint32_t nseg, n_sq, n_sq_lds, pat_off;
    uint32_t n_sieve;
    uint32_t n_bucket;  // primes with index in [n_bucket, n_sieve) reach the sieve through buckets
    uint32_t n_lane;    // bucketed primes from this index on have at most 64 multiples per block
    uint32_t n_sq_lane; // squares from this index on have at most 64 multiples per block
};

// One y-block [y1, y2] of the sweep.  The scalar fields below mirror *bp on
// the host (for grid sizes); kernels take the values from *bp.
struct BlockArgs {
    const BlockParams *bp;
    uint64_t y1, y2;
    uint32_t nseg;
    uint32_t n_small;   // primes with index in [FIRST_SIEVED, n_small) are < SMALL_P
    uint32_t n_sieve;   // primes with index < n_sieve are sieved (p <= max(sqrt(y2), SMALL_P))
    uint32_t n_sq_lds;  // primes with index < n_sq_lds have p <= SQ_LDS_P
    uint32_t n_sq;      // primes with index < n_sq have p^2 <= y2
    uint32_t n_sq_lane; // ... of which those from n_sq_lane on (p^2 > span / 64) take a lane each
    uint32_t n_bucket;  // primes with index in [n_bucket, n_sieve) (all > SEG) are bucketed
    uint32_t n_lane;    // ... of which those from n_lane on (> span / 64) are walked per lane
    uint32_t pat_off;   // y1 mod PAT
    uint2 *pres;              // {p, y1 mod p}: primes >= 5 ascending, residue per block
    uint64_t *res2;           // y1 mod p^2    (per block)
    const uint32_t *pat32;    // pattern bytes as words, length PAT_WORDS
    // per 32 y one 16-byte record {mu = +1 bits | mu = -1 bits << 32,
    // M(y) just before the record's first y (int64)}; 4 uint64 per 64 y
    uint64_t *words;
    // per segment: look-back state of the fused prefix scan, 2-bit flag
    // (1 = segment total, 2 = M(y) at the segment's end) over a 62-bit value
    uint64_t *seg_state;
    uint32_t *seg_ticket;     // segments are claimed in ticket order
    uint32_t *sq_cnt;         // per segment: large-square hits listed (may exceed SQ_BUCKET)
    uint32_t *sq_buf;         // per segment: SQ_BUCKET offsets of large-square multiples
    // bucketed primes: per (bucket workgroup, segment) counts, then offsets;
    // per segment first entry (nseg + 1); entries (offset in segment | log << 17)
    uint32_t *bk_cnt;
    uint32_t *bk_start;
    uint32_t *bk_buf;
    uint32_t *bk_stage;       // fill-pass entries per (group, workgroup) before regrouping
    uint64_t *bk_total;       // running count of bucket entries over blocks
    int64_t *carry;           // M(y1 - 1), advanced by the block's last segment
};

// The per-query state of one sweep (a batch of queries sharing the sieve).
struct QueryArgs {
    uint32_t nq;
    const uint64_t *q_n, *q_L, *q_g0;   // per query: n, L, first global x index
    // per global x index g (query q, x = g - q_g0[q] + 1)
    uint64_t *x_m, *x_Y, *x_K, *x_k0;  // m = n/x, Y, K (k part end), k0
    uint64_t *S;                        // wrapping uint64 contribution sums
    int64_t *A;                         // final M(floor(n/x))
    uint64_t *x_klo, *x_khi;            // k range of the current block
    // Queries with equal L form one keyed group when there are several:
    // its entries are the distinct pairs (x, m = floor(n_i/x)) over the
    // group's n_i, sorted by x then m (S and A depend on x and m only).
    const uint32_t *key_x;    // per entry of a keyed group: x
    const uint32_t *key_off;  // per group, x = 1..L+1: first entry of x (from the group's g0)
    const uint64_t *q_koff;   // per query: its group's base in key_off, or ~0 (plain query)
    // tiles: 64 consecutive x of one plain query (tile_x0 >= 1) or 64
    // consecutive entries of a keyed group (tile_x0 = 0)
    uint32_t ntiles;
    const uint32_t *tile_q, *tile_x0, *tile_nx;
    const uint64_t *tile_g0;
    uint64_t *tile_ymax;
    // per-block work description
    uint64_t *tile_klo, *tile_khi;
    uint32_t *tile_mode, *tile_nmu;
    uint64_t *tile_items;               // items per tile, then exclusive prefix (ntiles+1)
    uint32_t *counter;                  // persistent work counter
    uint64_t *pair_stats;               // [0] y-side visits, [1] k pairs, [2] run-length
                                        // pairs, [3] explicit-k pairs, [4] of those, the band's
    // Wide arguments (n >= 2^64): per query the high word of n and the number
    // xb of leading x whose m = floor(n/x) >= 2^wide_bits.  Those x take
    // the wide entries below (m in 128 bits); their plain slots do no work.
    const uint64_t *q_nhi, *q_xb;
    uint32_t w_n;                                    // wide entries
    const uint64_t *w_g;                             // per entry: global x index
    const uint32_t *w_x, *w_q;                       // x and query
    uint64_t *w_mlo, *w_mhi, *w_K, *w_Y, *w_k0;      // m (128 bits), K, Y, k0
    uint64_t *w_klo, *w_khi;                         // k range of the current block
    // tuning
    double beta;
    uint32_t ychunk, kchunk;
    uint32_t kbal;     // balanced runs where the 8 x 8 walk would use < 1/kbal of its lanes
    uint32_t rl_fast;  // 1: check-free fp64 floors where every m < 2^48
};

// ---------------------------------------------------------------- launchers
// All return the hipError_t of the launch (hipGetLastError()).
hipError_t launch_zero_u64(uint64_t *p, size_t n, hipStream_t s);
// *cur = p (direct launches)
hipError_t launch_block_set(const BlockParams &p, BlockParams *cur, hipStream_t s);
// *cur = table[*index]; ++*index (first node of the captured block graph)
hipError_t launch_block_next(const BlockParams *table, BlockParams *cur, uint32_t *index,
                             hipStream_t s);
hipError_t launch_plan(const QueryArgs &q, hipStream_t s);
hipError_t launch_block_setup(const BlockArgs &b, hipStream_t s);
hipError_t launch_square_buckets(const BlockArgs &b, hipStream_t s);
// multiples of the primes above SEG, sorted into per-segment buckets
// (events, if given, are recorded before the fill pass, between it and the
// regrouping pass, and after that)
hipError_t launch_prime_buckets(const BlockArgs &b, hipStream_t s, hipEvent_t fill0 = nullptr,
                                hipEvent_t fill1 = nullptr, hipEvent_t fill2 = nullptr);
hipError_t launch_sieve(const BlockArgs &b, hipStream_t s);
// per-block k ranges, -K M(Y) and item counts; with a band (wa < wb) the
// explicit-k chunks of band tiles skip the gap the band leaves
hipError_t launch_update_prep(const QueryArgs &q, const BlockArgs &b, hipStream_t s,
                              uint32_t wa = 0, uint32_t wb = 0);
// wide entries: plan (once per sweep), per-block k ranges and -K*M(Y), and
// the per-block run-length and explicit-k sums
hipError_t launch_wide_plan(const QueryArgs &q, hipStream_t s);
hipError_t launch_wide_prep(const QueryArgs &q, const BlockArgs &b, hipStream_t s);
hipError_t launch_wide_update(const QueryArgs &q, const BlockArgs &b, hipStream_t s);
hipError_t launch_scan_items(const QueryArgs &q, hipStream_t s);
// persistent update; explicit-k pairs with quotients in [2^wa, 2^wb) are
// left to launch_ek_window when wa < wb (wa = wb = 0: none)
hipError_t launch_update(const QueryArgs &q, const BlockArgs &b, uint32_t grid, hipStream_t s,
                         uint32_t wa = 0, uint32_t wb = 0);
// those pairs within the block, y-major over windows of 2^17 y covering
// [ystart, yend): ystart = max(2^wa, y1) a multiple of 2^17, yend =
// min(2^wb, y2 + 1) <= 2^31
hipError_t launch_ek_window(const QueryArgs &q, const BlockArgs &b, uint64_t ystart,
                            uint64_t yend, hipStream_t s);
// qlist = NULL finalizes queries 0..count-1, else the listed query indices
hipError_t launch_finalize(const QueryArgs &q, const uint32_t *qlist, uint32_t count,
                           hipStream_t s);
// level (lo, hi] of keyed group member qi's finalize (`entries` entries in
// it), gsz lanes per entry (a power of two up to 64)
hipError_t launch_finalize_keyed_level(const QueryArgs &q, uint32_t qi, uint64_t lo, uint64_t hi,
                                       uint64_t entries, uint32_t gsz, hipStream_t s);
hipError_t launch_collect(const QueryArgs &q, int64_t *out, hipStream_t s);
// out[c-1] = A entry of (c, floor(n_qi/c)) for c = 1..count (keyed group member qi)
hipError_t launch_keyed_byproducts(const QueryArgs &q, uint32_t qi, uint64_t count, int64_t *out,
                                   hipStream_t s);
// Interval sweep (records of the current block, relative to *off):
// *off = m_a - (record value at a)
hipError_t launch_interval_base(const BlockArgs &b, uint64_t a, int64_t m_a, int64_t *off,
                                hipStream_t s);
// running extremes of M(n)/sqrt(n) over n in [lo, hi] into part[IV_WGS][4]
// = {n_min, M(n_min), n_max, M(n_max)} (n = 0: none yet)
hipError_t launch_interval_extreme(const BlockArgs &b, uint64_t lo, uint64_t hi,
                                   const int64_t *off, uint64_t *part, hipStream_t s);
// dst[i] = M(lo + i) for i < count
hipError_t launch_interval_values(const BlockArgs &b, uint64_t lo, uint64_t count,
                                  const int64_t *off, int64_t *dst, hipStream_t s);
// res[0..3] = the reduced extremes of part, res[4] = M(n_end) (n_end in block b)
hipError_t launch_interval_final(const BlockArgs &b, const uint64_t *part, uint64_t n_end,
                                 const int64_t *off, int64_t *res, hipStream_t s);
hipError_t launch_debug_div(const uint64_t *n, const uint64_t *d, uint64_t *q, size_t count,
                            hipStream_t s);
hipError_t launch_debug_mu(const BlockArgs &b, uint64_t y_first, uint32_t count, int8_t *mu,
                           int64_t *mert, hipStream_t s);

// The 128-bit helpers of the wide entries on count arguments (out: two words
// each; op as in mertens_debug_wide), on the device and in a host build.
hipError_t launch_debug_wide(const uint64_t *mlo, const uint64_t *mhi, const uint64_t *d,
                             uint64_t *out, size_t count, int op, hipStream_t s);
void host_wide(int op, uint64_t mlo, uint64_t mhi, uint64_t d, uint64_t *qlo, uint64_t *qhi);

// acc += sum over y in the block, 1 <= y <= ymax, of w(y) M(y) mod 2^64 with
// w(y) = floor(n/y) - floor(n/(y+1)) (floor(n/ymax) - L at ymax)
hipError_t launch_debug_runsum(const BlockArgs &b, uint64_t nlo, uint64_t nhi, uint64_t ymax,
                               uint64_t L, uint64_t *acc, hipStream_t s);

// Host build of the device division routine (for tests without a GPU).
void host_magic(uint32_t d, uint64_t *mul, uint32_t *sh1, uint32_t *sh2);
uint64_t host_div(uint64_t n, uint64_t mul, uint32_t sh1, uint32_t sh2);

}  // namespace mrt
