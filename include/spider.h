/*
 * spider.h -- C ABI of the MI355X (gfx950) strided-swap stencil library.
 *
 * The library applies iterated 1-D / 2-D / 3-D stencils (SPIDER, Sec. 2.2: each
 * point becomes a weighted linear combination of its radius-r neighbourhood,
 * repeated over time steps, each step reading only the previous one) by
 * lowering every kernel row to a banded matrix product Y = K X (Sec. 3.1.1),
 * permuting the band's columns ahead of time with a strided swap so that every
 * group of four columns holds at most two non-zeros (Sec. 3.1.2, Fig. 5), and
 * permuting the input rows on the fly inside the register gather so the product
 * is unchanged (Sec. 3.2).  The product runs on the gfx950 structured-sparse
 * matrix instruction (v_smfmac_f32_16x16x64_{f16,bf16}) or, for comparison, on
 * the dense one (v_mfma_f32_16x16x32_{f16,bf16}); a plain direct-sum engine
 * serves fp32 / fp64 grids.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 *  - Every function returns a spider_status and never throws.  On failure a
 *    human-readable message is available from spider_last_error() (per thread).
 *  - Grids are interior-only, contiguous, row-major with x fastest:
 *    1-D grid[x], 2-D grid[y][x], 3-D grid[z][y][x]; `shape` lists extents slowest first.
 *    The halo is a fixed zero (Dirichlet-0) boundary of width r on every side.
 *  - Coefficients are fp64, (2r+1)^ndim of them, laid out w[dz][dy][dx] with
 *    each index 0..2r; w[o] multiplies x[p + o - r] (correlation, no flip).
 *  - Device pointers are plain HIP device addresses (e.g. from a PyTorch
 *    tensor's data_ptr()); `stream` is a hipStream_t passed as void* (NULL =
 *    the null stream).  The caller owns every buffer it passes in.
 *  - Work is asynchronous on `stream`: argument and launch errors are returned
 *    at once; device faults surface at the caller's next synchronisation.
 */
#ifndef SPIDER_H
#define SPIDER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPIDER_OK = 0,
    SPIDER_ERR_INVALID = 1,     /* bad argument (null pointer, size, radius, dtype...) */
    SPIDER_ERR_UNSUPPORTED = 2, /* valid request the library does not run (e.g. sparse fp32) */
    SPIDER_ERR_OOM = 3,         /* device or host allocation failed / over budget */
    SPIDER_ERR_HIP = 4,         /* a HIP runtime call failed */
    SPIDER_ERR_NOT_READY = 5,   /* ticket still running */
    SPIDER_ERR_BUSY = 6,        /* server queue full */
    SPIDER_ERR_CLOSED = 7       /* server shut down / ticket unknown */
} spider_status;

typedef enum { SPIDER_F64 = 0, SPIDER_F32 = 1, SPIDER_F16 = 2, SPIDER_BF16 = 3 } spider_dtype;

typedef enum {
    SPIDER_ENGINE_AUTO = 0,   /* sparse for 16-bit carries, direct otherwise */
    SPIDER_ENGINE_SPARSE = 1, /* strided swap + v_smfmac on 16-bit operands; the carry is the
                                 operand type, or fp32 with operands split from it */
    SPIDER_ENGINE_DENSE = 2,  /* same band and gather on dense v_mfma (16-bit operands) */
    SPIDER_ENGINE_DIRECT = 3  /* plain neighbour sum on the vector ALUs (fp32 / fp64 carries) */
} spider_engine;

/* Plan options.  Zero-initialise and set what you need; spider_opts_default fills defaults. */
typedef struct {
    int carry;     /* spider_dtype of the grids passed to apply (default SPIDER_F16) */
    int engine;    /* spider_engine (default AUTO) */
    int split;     /* products on the matrix engines (ignored by the direct engine):
                      1 = w rounded once to the operand type,
                      2 = w_hi + w_lo, each rounded (default),
                      3 = fp32 carry: also splits every input value x = x_hi + x_lo
                          and adds the products with x_lo (two instructions per kernel row);
                          a 16-bit carry on a 1-D line: the fused launches keep their
                          intermediate steps as such hi/lo pairs and round the grid to 16
                          bits once per launch instead of once per step (single-step
                          launches are those of split 2); other 16-bit grids: INVALID */
    int tile_h;    /* output rows per wavefront segment, 0 = chosen by the autotuner */
    int use_graph; /* 1 = capture each (in, out, steps) time loop of two or more launches
                      once as a hipGraph and replay it (default; a loop of one launch is
                      launched directly), 0 = launch every step */
    int autotune;  /* 1 = when tile_h is 0, time candidate segment heights on the device at
                      plan time and keep the fastest (results cached per shape, radius,
                      engine and dtype for the life of the process); 0 = occupancy heuristic */
    int time_block; /* time steps fused per launch, 0..16 (default 0 = automatic):
                       - paired-line bands with a 16-bit carry: up to four (the dense
                         engine three); automatic: four from 2^25 points, three from
                         2^23, else two;
                       - paired-line bands with an fp32 carry: up to three on the sparse
                         engine, two on the dense one; automatic: as above, capped;
                       - other 2-D grids of radius <= 3 on the matrix engines with a
                         16-bit carry: two;
                       - 1-D lines of radius <= 3 (16-bit or fp32 carry): up to four;
                         automatic: four from 2^22 points, else two;
                       - 3-D grids: two for radius 1 with a 16-bit carry, only when asked
                         for (measured slower on the 512^3 and 256^3 workloads);
                       - the direct engine on 2-D grids of radius <= 3: up to 16 steps
                         in LDS tiles of 32 x 32 outputs with a halo of T r points, at
                         most 64 points a side (radius 2: 8, radius 3: 5); automatic: the
                         most it allows on grids of up to 2^20 points (where single-step
                         launches are bound by latency), else one; bit-identical to
                         single steps;
                       - anything else: one.
                       Larger values are capped at the plan's maximum.  With 0 and
                       autotune the matrix-engine plans also time the depths and keep
                       the fastest per step.  A time loop of n steps runs n / T fused
                       launches, then (T > 2) one two-step launch for a remainder of two
                       or three steps, then a single step for one; the direct engine
                       runs its remainder as one launch.  The results agree to rounding;
                       on 1-D lines and on the direct engine they are identical bit for
                       bit, and see band_height for 2-D. */
    int operand;   /* matrix engines with an fp32 carry: 16-bit operand type, SPIDER_F16
                      (default, also when 0) or SPIDER_BF16.  With a 16-bit carry the operand
                      is the carry type and this field must be 0 or equal to it. */
    int band_height; /* output points per band row on the matrix engines: 0 = automatic
                        (8 where it applies, else 16), 16 = 16-point chunks with 32-column
                        windows (any radius), 8 = the paper's band height L = 2r + 2 <= 8
                        with two output lines per instruction (2-D, radius <= 3, 16-bit or
                        fp32 carry; segment heights are rounded up to even numbers).  The two
                        give different rounding orders.  With band height 8 and odd r, fused
                        steps (time_block >= 2) round differently from single steps; with
                        even r, or band height 16, they are identical bit for bit. */
    int row_swap;  /* where the input rows are swapped to match the strided-swapped kernel
                      matrix (Sec. 3.2): 0 = implicitly, in the gather's LDS offsets (default);
                      1 = explicitly, by copying each staged line into a swapped operand tile
                      in LDS first -- the comparison of the paper's Table 3, for measurement.
                      Same result bit for bit.  1 needs the sparse engine, a 16-bit carry, a
                      2-D grid and band height 16, and runs one step per launch (band_height
                      0 resolves to 16, time_block 0 to 1; other values are UNSUPPORTED);
                      batched apply and the server reject such plans. */
} spider_opts;

typedef struct spider_plan_s* spider_plan_t;
typedef struct spider_server_s* spider_server_t;

/* Fill `o` with the defaults listed above.  Returns SPIDER_ERR_INVALID if o is NULL. */
spider_status spider_opts_default(spider_opts* o);

/*
 * spider_plan: offline transformation (Sec. 3.1, done once per stencil; the paper
 * reports it as a small rule-based cost outside the timed loop, Sec. 4.2).
 *   coeffs  host fp64 array, (2r+1)^ndim, layout above; copied, not retained
 *   ndim    1, 2 or 3 (1-D lines run on the 16-point band engine, one to four steps
 *           per launch, or on the direct engine)
 *   shape   host array of ndim extents, each in [1, 2^31); a line (the last extent)
 *           may hold at most 2^30 - 1 bytes of state
 *   radius  1..7 (r = 7 is the largest radius the paper works through, Sec. 3.2)
 *   opts    NULL for defaults
 *   out     receives the plan handle
 * Builds, per kernel row with a non-zero tap, the banded matrix, pads it, applies
 * the strided column swap, splits coefficients into 16-bit hi/lo parts, compresses
 * to 2:4 values + 2-bit indices and packs them in the gfx950 lane order and uploads
 * them to the current HIP device.  A grid-sized scratch buffer is allocated on the
 * first spider_apply / spider_apply_batch (or at plan time when autotuning).
 * Errors: INVALID (arguments; on the matrix engines also a coefficient whose 16-bit
 * rounding overflows, |w| > 65504 for fp16), UNSUPPORTED (e.g. a matrix engine with an fp64 carry),
 * OOM, HIP.  The plan is immutable after
 * creation and owns its device memory.
 */
spider_status spider_plan(const double* coeffs, int ndim, const int64_t* shape, int radius,
                          const spider_opts* opts, spider_plan_t* out);

/*
 * spider_apply: out = S^steps(in) on `stream`: `steps` applications of the
 * stencil update of Sec. 2.2 (every point replaced by the weighted sum of its
 * radius-r neighbourhood), each step reading only the previous step's grid
 * (Jacobi), with the zero halo; each step is computed as the banded products of
 * Sec. 3.1.1 on the strided-swapped operands (Sec. 3.1.2, 3.2).
 *   in, out  device grids of the plan's shape in the plan's carry dtype; `in` is
 *            never written unless in == out (allowed); steps == 0 copies.
 *   steps    >= 0
 * The plan's scratch buffer holds intermediate steps, so two applies of one plan
 * must not overlap in time (use one plan per concurrent stream).
 * With use_graph, a loop of at most 512 launches is captured once per (in, out,
 * steps) as one graph and replayed; a longer loop replays one cached graph per
 * 256-launch body (so graphs stay bounded in size) and launches the remainder
 * directly.  The caches hold at most 64 and 16 graphs per plan; evicting one
 * waits for the device first.
 * Errors: INVALID (null plan/pointer, steps < 0, or a device other than the one
 * current at spider_plan is current), HIP (launch failure).
 */
spider_status spider_apply(spider_plan_t plan, const void* in, void* out, int steps, void* stream);

/*
 * spider_apply_noalloc: spider_apply without any device memory allocation, for
 * callers that cannot allocate (code under hipGraph capture, tight serving
 * loops, harnesses that forbid hipMalloc).
 *   Same arguments, semantics and results (bit for bit) as spider_apply, but the
 *   intermediate steps ping-pong through a fixed device array of
 *   SPIDER_NOALLOC_SCRATCH_BYTES bytes that the library holds on every GPU it
 *   runs on until the process ends, instead of the plan's own scratch buffer, and
 *   the loop's launches are enqueued directly (no graph is built).  The first
 *   call on a device looks the array's address up once (hipGetSymbolAddress).
 *   Every call on one GPU shares that GPU's array: calls that overlap in time on
 *   one GPU (from any plan, stream or thread) race and must not be issued.
 *   Nothing in the array needs clearing between calls.
 * Errors: INVALID (as spider_apply, and a grid larger than
 * SPIDER_NOALLOC_SCRATCH_BYTES), HIP (launch failure).
 */
#define SPIDER_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
spider_status spider_apply_noalloc(spider_plan_t plan, const void* in, void* out, int steps, void* stream);

/* Release the plan's device memory and cached graphs.  NULL is accepted. */
spider_status spider_plan_destroy(spider_plan_t plan);

/*
 * spider_plan_info: describe a plan (host query, no device work).
 *   engine, carry, tile_h (segment height of the one-step kernel), nrows_nonzero
 *   (kernel rows on the matrix path; for paired-line bands the r + 1 instructions
 *   per input line pair), scratch_bytes (size of the grid-sized scratch buffer the
 *   plan allocates on first use), time_block (steps fused per launch), tile_h2
 *   (segment height of the fused kernel, 0 if time_block is 1 and for the direct
 *   engine, whose fused kernel uses fixed 32 x 32 tiles), band_height (output
 *   points per band row: 16, or 8 for paired-line bands; 0 for the direct engine).
 *   Any output pointer may be NULL.
 */
spider_status spider_plan_info(spider_plan_t plan, int* engine, int* carry, int* tile_h,
                               int* nrows_nonzero, size_t* scratch_bytes, int* time_block,
                               int* tile_h2, int* band_height);

/*
 * spider_plan_work: what spider_apply(plan, in, out, steps) issues on the device
 * (host query, no device work), for measurement against the hardware's roofs.
 *   launches             kernel launches of the time loop (0 for steps == 0)
 *   matrix_instructions  matrix instructions of all of them (smfmac 16x16x64 on the
 *                        sparse engine, mfma 16x16x32 on the dense one; 0 for the
 *                        direct engine)
 * Either output pointer may be NULL.  With steps == time_block the loop is exactly
 * one launch of the plan's fused kernel.
 * Errors: INVALID (null plan, steps < 0), UNSUPPORTED (matrix_instructions asked
 * for a plan other than paired-line bands (any carry), a 1-D line, a 3-D grid at
 * one step per launch with a 16-bit carry, or the direct engine; *launches is still
 * set).
 */
spider_status spider_plan_work(spider_plan_t plan, int steps, uint64_t* launches, uint64_t* matrix_instructions);

/*
 * spider_measure_matrix_rate: the rate at which the current device sustains fp16
 * matrix instructions with register-resident operands and no memory traffic:
 * 2:4-sparse smfmac 16x16x64 (sparse = 1) or dense mfma 16x16x32 (sparse = 0).
 * Both do 16 x 16 x 32 multiply-adds per instruction; the sparse unit selects 2
 * of every 4 inputs first (Sec. 2.1), so the ratio of the two rates is the
 * speedup the sparse engine can bring here, and the sparse rate is the matrix
 * ceiling the stencil kernels run against at the same occupancy.
 *   waves_per_simd          1..4 resident waves per SIMD (one-wave workgroups)
 *   iterations              1..10^7; each wave issues 8 x iterations instructions
 *   stream                  hipStream_t as void* (NULL = default stream)
 *   dense_equiv_tflops      out: 2 x 16 x 16 x 32 flop per instruction / second
 *   clock_ghz               out (may be NULL): shader clock held meanwhile,
 *                           from the shader-cycle and 100 MHz real-time counters
 *   cycles_per_instruction  out (may be NULL): clock cycles per instruction per SIMD
 * Synchronous: allocates two small device buffers, runs a warm-up launch and a
 * timed one, frees the buffers.  Measurement only; no stencil state is touched.
 * Errors: INVALID (arguments out of range, null dense_equiv_tflops), OOM, HIP.
 */
spider_status spider_measure_matrix_rate(int sparse, int waves_per_simd, int iterations, void* stream,
                                         double* dense_equiv_tflops, double* clock_ghz,
                                         double* cycles_per_instruction);

/*
 * Batched apply (launches over the tiles of every grid).
 * Runs grids of uneven size and stencil shape together.  Grids whose plan uses a
 * matrix engine with a 16-bit carry, the implicit row swap and a 2-D radius of 1..3
 * or a 3-D radius of 1 are batched, one sequence of launches per (carry dtype,
 * engine): launch k advances every such grid that still has work, 2-D grids with
 * paired-line bands by two fused time steps per launch (steps[i] / 2 launches, then
 * one single step when steps[i] is odd), other grids by one step.  Each of their
 * results equals spider_apply of a plan with time_block = 2 bit for bit (one step
 * per launch where two cannot be fused; a plan fusing more steps agrees up to
 * rounding).  Every other plan (the direct engine, an fp32 carry, 1-D lines, larger
 * radii, the explicit row swap) runs its own time loop after them on the same
 * stream, exactly as spider_apply.
 *   n       number of grids, 1..4096
 *   plans, ins, outs, steps: host arrays of n entries, as for spider_apply.
 * Errors: INVALID (also: a plan of another device than the current one, or one plan
 * twice), OOM, HIP.
 */
spider_status spider_apply_batch(int n, const spider_plan_t* plans, const void* const* ins,
                                 void* const* outs, const int* steps, void* stream);

/* ------------------------------------------------------------------ serving */

/*
 * spider_server_create: start a continuous-batching request loop on the
 * current HIP device.  Requests are admitted while their device footprint
 * (two grid-sized buffers of the plan's carry dtype) fits in `hbm_budget_bytes`
 * and a slot is free (max_slots); admitted requests share every round's
 * batched launch (2-D grids whose plan fuses three or four steps, and plans that
 * batched apply runs alone, run their own launches in the round instead), and a
 * request that arrives while others run joins at the next round.  Grid state
 * stays on the device between rounds.  Any plan spider_apply accepts is accepted.
 */
spider_status spider_server_create(size_t hbm_budget_bytes, int max_slots, int max_queue,
                                   spider_server_t* out);

/*
 * spider_submit: enqueue out = S^steps(in) for `plan`.  `in` and `out` are
 * device buffers owned by the caller, and `plan` a plan owned by the caller;
 * all three must stay valid (not freed, not destroyed) until spider_poll has
 * reported the ticket done, or until spider_server_destroy has returned.  `in`
 * is read once at admission.  Returns BUSY if the queue is full, OOM if the
 * request alone exceeds the budget, INVALID on bad arguments or a plan built
 * on another device than the server's.  A request whose scratch buffer cannot
 * be allocated while no other request runs completes with OOM.
 */
spider_status spider_submit(spider_server_t srv, spider_plan_t plan, const void* in, void* out,
                            int steps, uint64_t* ticket);

/*
 * spider_poll: *done = 1 once the result is in `out` (then *result holds its
 * status).  A ticket reported done is released: polling it again returns CLOSED
 * (unknown ticket).  Tickets that are never polled are released by
 * spider_server_destroy.
 */
spider_status spider_poll(spider_server_t srv, uint64_t ticket, int* done, spider_status* result);

/*
 * spider_server_stats: latency of completed requests in microseconds (submit ->
 * result written), percentiles over the most recent 65536 successful
 * completions, the number of successful completions and the stencil updates
 * (points x steps) they performed.
 */
spider_status spider_server_stats(spider_server_t srv, double* p50_us, double* p99_us,
                                  uint64_t* completed, double* stencil_updates);

/* Stop the loop: finishes admitted requests, fails queued ones with CLOSED, frees memory. */
spider_status spider_server_destroy(spider_server_t srv);

/* ------------------------------------------------------------------ host-side introspection
 * These run on the host only (no HIP call); they expose the offline transformation
 * so it can be checked without a GPU.
 */

/*
 * spider_gather_positions: window position of every K slot of one 32-column band
 * as the gfx950 gather reads it.  pos[k], k = 0..31, is the band column (0..31)
 * whose input row feeds slot k; a permutation of 0..31.  The band of an output
 * chunk of 16 points at x0 covers input columns x0-8 .. x0+23.
 */
spider_status spider_gather_positions(int pos[32]);

/*
 * spider_swap_columns: the strided column swap of Sec. 3.1.2 on an L x 2L band
 * (Fig. 5 stage 2): perm[j] = original column now at column j, j = 0..2L-1.
 *   granularity 1: element columns, odd j < L exchanged with j + L (the paper's rule)
 *   granularity 2: the same rule on pairs of columns (32-bit units of 16-bit data)
 * Errors: INVALID for L < 2, L odd, or granularity not 1/2 (L must be even for 2).
 */
spider_status spider_swap_columns(int L, int granularity, int* perm);

/*
 * spider_compress_24: 2:4 compression of a rows x cols matrix (cols % 4 == 0) whose
 * every group of 4 has at most 2 non-zeros (Fig. 5 stage 3).  vals is rows x cols/2,
 * meta is rows x cols/2 2-bit positions (one byte each, 0..3), increasing within a
 * group; a group with one non-zero keeps a zero placeholder at the next position
 * (at position 2 if the non-zero is at 3), an all-zero group uses positions 0, 1.
 * Errors: INVALID if a group holds more than 2 non-zeros or sizes are bad.
 */
spider_status spider_compress_24(const double* m, int rows, int cols, double* vals, uint8_t* meta);

/*
 * spider_pack_row: the packed smfmac operands of one kernel row as the 2-D/3-D
 * kernels load them.  row: 2r+1 fp64 taps along x; operand SPIDER_F16/BF16; split 1/2.
 *   a_bits  64 lanes x 8 16-bit values (compressed A of the 16 x 64 operand
 *           [K'_hi | K'_lo], lane-major)
 *   idx     64 lanes x 16-bit index field (2 bits per compressed value)
 *   dense_bits  64 lanes x 16 16-bit values: dense A of K'_hi (8) then K'_lo (8), or NULL
 * Errors: INVALID.
 */
spider_status spider_pack_row(const double* row, int radius, int operand, int split, uint16_t* a_bits,
                              uint16_t* idx, uint16_t* dense_bits);

/*
 * spider_pair_gather_positions: window column of every K slot of one line's
 * 16-slot block in the paired-line band (2-D, r <= 3; the paper's band height
 * L = 2r + 2 rounded to 8 with two output lines stacked, Sec. 3.1.2 and Eq. 1).
 * pos[s], s = 0..15, is a permutation of 0..15; the window of an 8-point output
 * chunk at x0 covers input columns x0-4 .. x0+11.
 */
spider_status spider_pair_gather_positions(int pos[16]);

/*
 * spider_pack_pair: the packed operands of instruction k (0..r) of the
 * paired-line band for a 2-D stencil.  w: (2r+1)^2 fp64 taps [dy][dx], r in 1..3;
 * operand SPIDER_F16/BF16; split 1/2.  The instruction's 16 x 64 operand has row
 * 8*phi + m (output line i + phi, point m of the chunk) and K slot
 * 32*lambda + 16*rho + s (input line j + lambda, rho = 0 hi / 1 lo coefficient
 * part, window column pos[s]); it holds kernel row 2k + lambda - phi, for input
 * pairs with j - i = 2k - r.
 *   a_bits      64 lanes x 8 16-bit values (compressed A, lane la: row la % 16,
 *               K slots 16*(la/16) .. +15)
 *   idx         64 lanes x 16-bit index field (2 bits per compressed value)
 *   dense_bits  64 lanes x 16 16-bit values: K slots 8*(la/16)+e of line j (8),
 *               then of line j + 1 (8), or NULL
 * Errors: INVALID.
 */
spider_status spider_pack_pair(const double* w, int radius, int operand, int split, int k, uint16_t* a_bits,
                               uint16_t* idx, uint16_t* dense_bits);

/* Message of the last failing call on this thread ("" if none). */
const char* spider_last_error(void);

/* Library version string. */
const char* spider_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPIDER_H */
