/*
 * mertens.h -- C ABI of the MI355X (gfx950) exact Mertens-function library.
 *
 * Computes M(n) = sum_{y<=n} mu(y) exactly for 0 <= n < 2^64 by the blocked
 * method of Kuznetsov, "Computing the Mertens function on a GPU"
 * (arXiv:1108.0135), Section 2 (identity and blocking) and Section 3
 * (segmented Moebius block sieve, per-block contribution update, finalize).
 * Every step of the computation runs in HIP kernels on one GPU; this header
 * uses plain C types only (no HIP or PyTorch types in any signature).
 *
 * Conventions shared by every entry point:
 *   - Return value 0 on success, or a negative errno-style code:
 *       MERTENS_EINVAL   bad argument (null pointer with count > 0, bad block
 *                        size, u too small for some n, ...)
 *       MERTENS_ENOMEM   device or host allocation failed; nothing written
 *       MERTENS_ENODEV   no usable GPU, or the context is not initialised
 *       MERTENS_ERANGE   index out of range (byproducts)
 *       MERTENS_EIO      a HIP runtime call or kernel launch failed
 *       MERTENS_EAGAIN   no free slot (serving)
 *       MERTENS_EINPROGRESS  result not ready yet (serving)
 *     mertens_strerror() turns a code into text; mertens_last_error() returns
 *     the text of the last failure with detail (file/line of the HIP call).
 *   - Pointers are HOST pointers unless stated otherwise; the caller owns
 *     them and the library never keeps them past the call.
 *   - No call is thread-safe: one context per process, one owner thread.
 *   - Results are exact integers (no tolerance); identical bits whatever the
 *     block size, u, tiling or batch composition.
 */
#ifndef MERTENS_H
#define MERTENS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MERTENS_EINVAL (-22)
#define MERTENS_ENOMEM (-12)
#define MERTENS_ENODEV (-19)
#define MERTENS_ERANGE (-34)
#define MERTENS_EIO (-5)
#define MERTENS_EAGAIN (-11)
#define MERTENS_EINPROGRESS (-115)

/*
 * mertens_init -- create (or re-create) the process-wide context on the
 * current HIP device.
 *   u      sieve limit used to split each query (Section 2: an array of
 *          floor(n/u) entries A[x] = M(floor(n/x)) is built while M(y) is
 *          sieved for y < u).  0 = automatic: about (sum of the batch's n)^(2/3).
 *          A query n uses L = max(1, floor(n/u)) entries; L must stay below
 *          2^31 (else mertens_query returns MERTENS_EINVAL).
 *   block  y-block length of the sieve sweep (Section 3: y is processed in
 *          blocks, in increasing order).  0 = automatic (2^30, or less when
 *          the sweep is shorter).  Otherwise a multiple of 2^17 in
 *          [2^17, 2^31].
 * Returns 0, MERTENS_EINVAL (bad block), MERTENS_ENODEV, MERTENS_ENOMEM.
 * Calling it again frees the previous context first.
 */
int mertens_init(uint64_t u, uint64_t block);

/*
 * mertens_query -- synchronous exact M(n[i]) for i < count.
 *   n     host array of count arguments (any order, duplicates allowed,
 *         0 <= n < 2^64; M(0) = 0 by convention, the empty sum).
 *   out   host array of count int64 results, written only on success.
 * All arguments of one call share one sieve sweep (Section 2: one sieve
 * serves several close values of n), each with its own A array.  The A
 * arrays stay on the device until the next query for mertens_byproducts().
 * Returns 0, MERTENS_EINVAL, MERTENS_ENOMEM, MERTENS_ENODEV, MERTENS_EIO.
 * count == 0 returns 0 and touches nothing.
 */
int mertens_query(const uint64_t *n, size_t count, int64_t *out);

/*
 * mertens_query_noalloc -- mertens_query for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * mertens_query, but every device buffer of the call (records, residues,
 * prime table, pattern copy, per-query arrays) is a piece of one static
 * 64 MiB device array that each GPU holds from library load until the
 * process ends; the call makes no hipMalloc or hipFree.  It sweeps in
 * blocks of at most 2^25 y with the sieve in turn (no graph, no sieve
 * ahead).  A request that needs more than the scratch holds (roughly, L and
 * the sieve bound of queries past 10^16) returns MERTENS_ENOMEM with
 * mertens_last_error() saying so, and nothing is written.  Calls on one
 * GPU share the scratch and must not overlap (they race; the library is
 * not thread-safe anyway); it is refused while the serving worker runs.
 * The A arrays are not kept: mertens_byproducts still refers to the last
 * mertens_query / mertens_query_wide.  Requires mertens_init.
 */
int mertens_query_noalloc(const uint64_t *n, size_t count, int64_t *out);

/*
 * mertens_query_wide -- mertens_query for arguments up to 2^96:
 * n[i] = n_hi[i] 2^64 + n_lo[i] with n_hi[i] < 2^32 (Section 5 computes
 * M(n) for n up to 10^22, past the 64-bit limit, with 128-bit integers).
 *   n_lo, n_hi  host arrays of count words; out as in mertens_query.
 * The x whose m = floor(n/x) needs more than 64 bits (x <= n / 2^64) get
 * 128-bit entries of their own: K = max(k0 - 1, floor(beta sqrt(m)),
 * floor(m / 2^32)) keeps Y = floor(m/(K+1)) below 2^32, so each run-length
 * quotient is three 32-bit digit steps and each explicit-k quotient is an
 * fp64 estimate with one exact 128-bit correction; every other x takes the
 * plain path.  Arguments with n_hi = 0 behave exactly as in mertens_query,
 * except that a batch holding any wide argument forms no keyed groups.
 * The sieve bound n/(L+1) must stay below 2^50 (automatic u keeps it far
 * lower).  Byproducts are available as after mertens_query.
 * Returns 0, MERTENS_EINVAL (null pointer, n_hi >= 2^32, u out of range),
 * MERTENS_ENOMEM, MERTENS_ENODEV, MERTENS_EIO.
 */
int mertens_query_wide(const uint64_t *n_lo, const uint64_t *n_hi, size_t count, int64_t *out);

/*
 * mertens_byproducts -- the other entries of query i's array from the last
 * successful mertens_query (Section 1: one evaluation at n yields every
 * M(floor(n/c)); the array holds them for c <= L = max(1, floor(n/u))).
 *   i     index into the last query's n[] array
 *   buf   host array of cap entries; buf[c-1] = M(floor(n_i/c)) for
 *         c = 1 .. min(L, cap)
 *   len   receives L (may be NULL)
 * Returns 0, MERTENS_ERANGE (i >= last count), MERTENS_EINVAL (buf NULL with
 * cap > 0), MERTENS_ENODEV, MERTENS_EIO.
 */
int mertens_byproducts(size_t i, int64_t *buf, size_t cap, size_t *len);

/*
 * Serving: asynchronous queries merged into one running sieve sweep.
 *
 * mertens_submit -- enqueue M(n) and return a ticket.  A worker thread of
 * the library runs a cyclic sweep over y-blocks; queued requests join it at
 * the next block boundary as a batch (admitted while the x entries in
 * flight, 64 B of device memory each, stay within "serve_x_budget"), so
 * requests that arrive while others are on the GPU share the sieve with
 * them (Section 2: one sieve serves several values of n).  Each query uses
 * u = n^(2/3) (or the u given to mertens_init) and completes as soon as
 * every block it needs has been visited once since it joined.  Results are
 * bit-identical to mertens_query.
 *   n       0 <= n < 2^64 (n = 0 completes at once with M(0) = 0)
 *   ticket  receives the request id
 * Returns 0, MERTENS_EAGAIN (already "serve_capacity" requests in flight),
 * MERTENS_EINVAL (ticket NULL), MERTENS_ENODEV, or the error that stopped
 * the worker (MERTENS_EIO / MERTENS_ENOMEM).
 *
 * mertens_poll -- result of a ticket.  Returns 0 and writes *out = M(n) and
 * *latency_s = seconds from submit to completion (either pointer may be
 * NULL; the ticket is then released), MERTENS_EINPROGRESS while pending,
 * MERTENS_ERANGE for an unknown or already collected ticket, or the error
 * that stopped the worker.
 *
 * The worker uses its own stream and device buffers; mertens_query may be
 * called meanwhile.  mertens_init and mertens_shutdown stop the worker and
 * drop uncollected tickets.
 */
int mertens_submit(uint64_t n, uint64_t *ticket);
int mertens_poll(uint64_t ticket, int64_t *out, double *latency_s);

/*
 * mertens_set_stream -- run all further device work on the given HIP stream
 * (a hipStream_t passed as void*; NULL = the library's own stream).  The
 * caller keeps ownership and must keep it alive while the context uses it.
 * Returns 0 or MERTENS_ENODEV.
 */
int mertens_set_stream(void *hip_stream);

/*
 * mertens_set_param -- tuning knobs (results never depend on them).
 *   "u_scale"     automatic u = u_scale * (sum of the batch's n)^(2/3), where
 *                 n within a relative 2^-20 of each other count once (they
 *                 share their update work); default 0.5
 *   "beta"        split of the per-x sum between the run-length part over
 *                 y <= Y and the explicit k part (K = floor(beta*sqrt(m))),
 *                 in (0, 1]; default 0.25
 *   "ychunk"      y per work item of the run-length part, multiple of 64
 *                 in [64, 2^20] (default 16384)
 *   "kchunk"      k per work item of the explicit k part (default 1024)
 *   "kbal"        explicit-k tiles whose 8 x 8 walk would keep fewer than
 *                 1/kbal of its lanes busy take balanced per-lane runs of
 *                 their pairs instead (default 0: never)
 *   "waves_per_cu" persistent update grid size per compute unit (default 12,
 *                 the waves of three resident workgroups)
 *   "block_auto"  y-block length when mertens_init got block = 0 (a multiple
 *                 of 2^17 in [2^17, 2^31]; default 2^30, or the whole sweep
 *                 when it is shorter)
 *   "graph"       1: replay one captured hipGraph of the per-block kernel
 *                 sequence; 0: direct launches (default)
 *   "sieve_ahead" direct launches: most blocks sieved ahead of the update on
 *                 a second stream, each holding B/2 bytes of records
 *                 (default 4; 1 = strictly in turn)
 *   "update_window" blocks starting below 2^30 are updated in windows of
 *                 2^update_window y so that the random M(y) reads of one
 *                 window stay cache-resident (17..40; default 0: whole
 *                 blocks)
 *   "bucket_min"  a block sieving at least this many primes above 2^17
 *                 lists their multiples in per-segment buckets first
 *                 (default 2^20; scanning them per segment is faster below);
 *                 a block also buckets them when they outnumber the
 *                 multiples they leave in a 2^17-y segment eight times or
 *                 more (from y near 1.5e13 on)
 *   "rl_fast"     1 (default): run-length quotients with m < 2^48 take the
 *                 test-free rounded-up fp64 floor, and explicit-k quotients
 *                 of such x the test-free fused form; 0: always the tested
 *                 path (and no band, below)
 *   "band_lo", "band_hi"  explicit-k pairs whose M(y) read has y in
 *                 [2^band_lo, 2^band_hi) are summed y-major: each window of
 *                 2^17 y of the block's records is staged in LDS once and
 *                 read there by every x with quotients in it (band_lo 0, or
 *                 17..30; band_hi up to 31; default [2^20, 2^28)); band_lo = 0
 *                 turns it off.  Applies with direct launches only.
 *   "progress"    k > 0: a query waits for every k-th block and prints
 *                 "mertens: block i of n updated" on stderr, and for each
 *                 update window of a block ("update_window") prints one line
 *                 per window (default 0: off)
 *   "wide_bits"   x with floor(n/x) >= 2^wide_bits take the 128-bit wide
 *                 entries of mertens_query_wide (33..64; default 64, i.e.
 *                 only those past 64 bits; lower values route more x there,
 *                 for testing, and disable keyed groups)
 *   "serve_capacity"  most requests in flight for mertens_submit (4096)
 *   "serve_x_budget"  most x entries of admitted requests (2^26 = 4 GiB)
 *   "serve_short_blocks" S: requests are served in six lanes by the number
 *                 of y-blocks their sweep needs (up to S, 4S, 16S, 64S, 256S,
 *                 more), each lane its own cyclic sweep, one block of every
 *                 busy lane per worker step (default 4)
 * Returns 0 or MERTENS_EINVAL (unknown key, value out of range, or a
 * non-serving key while the serving worker runs).
 */
int mertens_set_param(const char *key, double value);

/*
 * mertens_get_param -- the current value of a mertens_set_param key into
 * *value, and "tuned": 1 when mertens_init applied the stored autotuner
 * choice (tuned_<arch>.json next to the library, taken on the kernel
 * sources this library was built from; the environment variable
 * MERTENS_TUNED=0 skips it), else 0.  mertens_init restores the built-in
 * defaults, then applies that file.
 * Returns 0, or MERTENS_EINVAL for an unknown key or a NULL pointer.
 */
int mertens_get_param(const char *key, double *value);

/*
 * mertens_stats -- counters of the last mertens_query or mertens_interval (benchmarking).
 * Writes up to cap doubles into vals in this order (returns how many):
 *   0 sieved y (Ymax+1)   1 blocks         2 u used        3 sum of L
 *   4 sum over x of Y (run-length range)  5 sum over x of explicit k terms
 *   6 ms sieve kernels (with the fused M(y) prefix)
 *   7 ms separate scan passes (none: always 0)  8 ms update prep  9 ms update
 *  10 ms finalize         11 ms total device time          12 update launches
 *  13 sieve launches      14 run-length quotients taken (mu(y) != 0, y <= Y)
 *  15 explicit k quotients taken (= M(y) gathers)
 *  16 bucket entries listed    17 ms bucket fill pass    18 bucketed prime visits
 *  19 ms bucket regrouping pass   (16-19: mertens_interval only, 0 after a query)
 *  20 ms of the y-major band kernel (part of 9)
 *  21 explicit k quotients taken by it (part of 15)
 * Kernel times are HIP-event intervals on the library's stream.
 */
int mertens_stats(double *vals, int cap);

/* mertens_shutdown -- free the context and every device buffer. */
void mertens_shutdown(void);

/* mertens_strerror -- static text for a return code. */
const char *mertens_strerror(int code);

/* mertens_last_error -- detail text of the last failure in this process. */
const char *mertens_last_error(void);

/*
 * mertens_interval -- every M(n) for n in [a, b] from one exact value, and
 * where M(n)/sqrt(n) is smallest and largest there (Section 6: once M is
 * known exactly at grid points, the gaps between them are covered by direct
 * sieving and the local extreme is read off the values).
 *   a, b    1 <= a <= b <= 2^64 - 2^32.
 *   m_a     M(a) if the caller knows it (e.g. from an earlier mertens_query),
 *           else NULL: the library first runs mertens_query on a, which
 *           replaces the arrays mertens_byproducts reads.
 *   m_b     out: M(b) (may be NULL).
 *   n_ext   out (may be NULL): n_ext[0] = the n in [a, b] with the smallest
 *           M(n)/sqrt(n), n_ext[1] = the n with the largest; equal ratios
 *           give the smaller n.  The comparison is exact (integer products,
 *           no rounding).
 *   m_ext   out (may be NULL): M(n_ext[0]), M(n_ext[1]).
 *   values  out (may be NULL): M(n) for n = a..b into values[0..b-a]; needs
 *           cap >= b - a + 1 and b - a + 1 <= 2^28.
 * The sweep sieves mu over [a - (a mod 2^17), b] in blocks (the init block
 * size, or automatically up to 2^31 y; device primes up to ceil(sqrt(b)),
 * those above 2^17 through per-segment buckets once there are "bucket_min"
 * of them or eight per multiple in a segment), runs the M(y) prefix from
 * zero, and shifts it by M(a) minus the
 * prefix at a.
 * mertens_stats afterwards: sieved_y, blocks, ms_sieve (the sieve kernel
 * with its fused prefix), ms_prep (block set-up, square and prime buckets),
 * ms_update (the interval reductions), ms_total, sieve_launches and slots
 * 16-19 (bucket entries, fill-pass ms, bucketed prime visits, regrouping
 * ms); others 0.
 * Returns 0, MERTENS_EINVAL, MERTENS_ENOMEM, MERTENS_ENODEV, MERTENS_EIO.
 */
int mertens_interval(uint64_t a, uint64_t b, const int64_t *m_a, int64_t *m_b, uint64_t *n_ext,
                     int64_t *m_ext, int64_t *values, size_t cap);

/*
 * Diagnostics used by the test suite.
 *
 * mertens_debug_div -- exact floor(n[i] / d[i]) for d[i] in [1, 2^32) by the
 * Granlund-Montgomery multiply-high method ("Division by invariant integers
 * using multiplication", PLDI 1994, Fig. 4.1), the replacement for 64-bit
 * hardware division that Section 3 asks for.  on_device = 0 runs the host
 * build of the same routine (no GPU needed), 1 runs it in a kernel.
 * Returns 0, MERTENS_EINVAL (d == 0 or d >= 2^32), MERTENS_ENODEV, MERTENS_EIO.
 */
int mertens_debug_div(const uint64_t *n, const uint64_t *d, size_t count,
                      uint64_t *q, int on_device);

/*
 * mertens_debug_wide -- the 128-bit quotient routines of mertens_query_wide on
 * count arguments m = m_hi 2^64 + m_lo and divisors d, into q_hi 2^64 + q_lo:
 *   op 0  floor(m/d), one quotient bit per step (any m, 1 <= d < 2^64)
 *   op 1  floor(m/d) mod 2^64 (q_hi = 0) by three 32-bit digit steps, each
 *         an fp64 estimate and one integer correction (m < 2^96, d < 2^32)
 *   op 2  floor(m/d) (q_hi = 0) by an fp64 estimate and an exact 128-bit
 *         check (floor(m/d) < 2^50)
 * on_device = 0 runs the host build of the same routines, 1 runs them in a
 * kernel.  Returns 0, MERTENS_EINVAL (null pointer, bad op, d = 0, or an
 * argument outside the op's range), MERTENS_ENODEV, MERTENS_EIO.
 */
int mertens_debug_wide(const uint64_t *m_lo, const uint64_t *m_hi, const uint64_t *d,
                       size_t count, uint64_t *q_lo, uint64_t *q_hi, int op, int on_device);

/*
 * mertens_debug_runsum -- for n = n_hi 2^64 + n_lo (< 2^82) and L >= 1, the
 * sum over k > L of M(floor(n/k)) mod 2^64 (the term S[1] of the identity
 * with split L, Section 2), evaluated the plain way: a sieve sweep over
 * y <= floor(n/(L+1)) (< 2^50) adding (floor(n/y) - floor(n/(y+1))) M(y),
 * with floor(n/ymax) - L at the top, and no explicit-k part.  With the
 * byproducts A[2..L] of a query using the same L it gives an independent
 * M(n) = 1 - S - sum A[k].  Slow (two quotients per y); "progress" reports.
 * Returns 0, MERTENS_EINVAL, MERTENS_ENODEV, MERTENS_ENOMEM, MERTENS_EIO.
 */
int mertens_debug_runsum(uint64_t n_lo, uint64_t n_hi, uint64_t L, uint64_t *s_out);

/*
 * mertens_debug_primes -- the host prime table the sieve uploads: the count,
 * the largest and the sum of the primes p with 5 <= p <= limit (limit <=
 * 2^32; segmented sieve of Eratosthenes over odd numbers).  Needs no GPU.
 * Returns 0 or MERTENS_EINVAL.
 */
int mertens_debug_primes(uint64_t limit, uint64_t *count, uint64_t *last, uint64_t *sum);

/*
 * mertens_debug_mu -- mu(y) for y in [y1, y1 + count) from the device sieve
 * (Section 3, the 8-bit log-prime sieve with the corrected log rule) into
 * the host array mu (int8), and, if mert != NULL, the window partial sums
 * mert[i] = sum_{z=y1}^{y1+i} mu(z) read back through the device prefix
 * scan (for y1 = 0 these are M(i)).  y1 + count <= 2^63, count <= 2^31.
 * Uses a sweep of its own; does not disturb the last query's byproducts.
 * Returns 0, MERTENS_EINVAL, MERTENS_ENOMEM, MERTENS_ENODEV, MERTENS_EIO.
 */
int mertens_debug_mu(uint64_t y1, size_t count, int8_t *mu, int64_t *mert);

#ifdef __cplusplus
}
#endif

#endif /* MERTENS_H */
