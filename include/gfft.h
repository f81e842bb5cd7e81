/*
 * gfft: one GPU's share of a slab-decomposed 3D real FFT on AMD Instinct
 * MI355X (gfx950).
 *
 * The method is the slab algorithm of Verma et al., "Scalable Multi-node
 * Fast Fourier Transform on GPUs" (section 3): a real N^3 field is split
 * into x-slabs of X = N/p planes; each GPU runs a 2D real-to-complex FFT
 * over (y, z) on its planes (step 1), reorders the result into p contiguous
 * chunks of (N/p) x (N/p) x (N/2+1) complex values for the all-to-all
 * exchange (steps 2-4), and finishes with a strided batched 1D complex FFT
 * along x (step 5).  The inverse runs the same steps in reverse order.  The
 * transforms are the unnormalized DFTs of section 2; because the field is
 * real only kz = 0..N/2 is stored (FFTW convention, K = N/2 + 1).
 *
 * Conventions used by every entry point
 *   - Arrays are C order, z fastest, x slowest.  A real grid is [X][N][N];
 *     its half spectrum is [X][N][K]; complex values are interleaved
 *     (re, im) pairs of the plan's real type.  A plan with batch B > 1
 *     processes B independent grids stored back to back.
 *   - All array pointers are DEVICE pointers owned by the caller, aligned to
 *     at least 16 bytes.  The library never allocates, frees, copies to the
 *     host or synchronizes inside an exec call; it only enqueues kernels on
 *     `stream` (a hipStream_t; NULL means the null stream).
 *   - Every argument is checked on the host before any HIP call, and every
 *     call returns a gfft_status; nothing is thrown and nothing aborts.  A
 *     failed kernel launch returns GFFT_E_HIP.  Errors raised while a kernel
 *     runs are reported by the caller's next synchronization.
 *   - Plans are immutable after creation: concurrent exec calls on one plan
 *     are safe when they use different streams and disjoint buffers.
 */
#ifndef GFFT_H
#define GFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GFFT_OK = 0,
    GFFT_E_INVALID_ARG = -1, /* NULL pointer, bad sign, aliasing, bad enum  */
    GFFT_E_UNSUPPORTED = -2, /* size/flag combination not supported         */
    GFFT_E_ALIGN = -3,       /* a data pointer is not 16-byte aligned       */
    GFFT_E_NOMEM = -4,       /* plan tables could not be allocated          */
    GFFT_E_HIP = -5,         /* a HIP runtime call or kernel launch failed  */
    GFFT_E_NO_DEVICE = -6,   /* no usable gfx950 device is present          */
    /* Not a status: widens the enumeration to every 32-bit value, so that
     * any int a caller passes where a gfft_status is expected (for example
     * to gfft_status_string) is a valid value of the type in C++ as in C. */
    GFFT_STATUS_MAX_ENUM = 0x7fffffff
} gfft_status;

typedef enum {
    GFFT_F64 = 0,
    GFFT_F32 = 1,
    /* Not a type: makes every 32-bit value a valid gfft_dtype, so that a bad
     * value reaches the argument check (GFFT_E_INVALID_ARG). */
    GFFT_DTYPE_MAX_ENUM = 0x7fffffff
} gfft_dtype;

/* Plan flags. */
enum {
    /* Slab plans: exec_r2c leaves the half spectrum in all-to-all send order
     * [p][X][N/p][K] (chunk j = wavenumbers ky in [j N/p, (j+1) N/p), one
     * chunk per destination rank, section 3 steps 2-3), and exec_c2r reads
     * that order.  The reorder is folded into the z pass's stores/loads, so
     * it costs no extra pass. */
    GFFT_FUSE_PACK = 1u << 0,
    /* FP32 plans, N >= 32: run the first radix-16 stage of the y and x passes
     * on the matrix cores as a real 32x32 GEMM (v_mfma_f32_32x32x16_bf16)
     * with every FP32 operand split into 2 (or 3) BF16 terms and FP32
     * accumulation.  A precision/speed variant of the FP32 vector path:
     * relative error per product about 2^-16 (2 terms) or 2^-24 (3 terms).
     * At most one of the two; GFFT_E_UNSUPPORTED for FP64 or N < 32. */
    GFFT_MFMA_BF16X2 = 1u << 1,
    GFFT_MFMA_BF16X3 = 1u << 2,
    /* In-place transforms in the FFTW padded layout (the paper counts
     * Nx/p x Ny x (Nz/2+1) points per GPU before step 1 and shares one work
     * space between R2C, C2C and C2R, section 3): every real row of N values
     * is padded to N + 2, so a real row and its K complex bins occupy the
     * same bytes.  exec_r2c / exec_c2r (and the adjoints and z passes) then
     * take the SAME pointer for the real and the complex argument, and the
     * grid needs half the memory.  Not combinable with GFFT_FUSE_PACK (the
     * send order moves rows); GFFT_E_UNSUPPORTED then. */
    GFFT_INPLACE = 1u << 3,
    /* Slab plans: use the paper's chunk order as the exchange wire format.
     * Step 2 (section 3) transposes the slab to [N][X][K] (ky slowest), so
     * chunk j is [N/p][X][K] = [ky_l][x_l][kz]; the send buffer is
     * [p][N/p][X][K] (the standalone pack, or exec_r2c with GFFT_FUSE_PACK).
     * gfft_exec_x_c2c then takes the received buffer [p][N/p][X][K]
     * (chunk i from rank i) and folds the chunk transpose of step 4 into its
     * addressing: line (ky_l, kz) has x = i X + x_l; its result stays in that
     * buffer order.  GFFT_E_UNSUPPORTED for full-grid plans. */
    GFFT_PACK_PAPER_ORDER = 1u << 4
};

typedef struct gfft_plan gfft_plan;

/* Byte sizes of the caller-owned buffers a plan works on. */
typedef struct {
    int64_t n;             /* grid edge N                                  */
    int64_t slab_x;        /* X = local x-planes                           */
    int64_t ranks;         /* p = N / X                                    */
    int64_t batch;         /* independent grids                            */
    int64_t k;             /* K = N/2 + 1                                  */
    int64_t real_bytes;    /* batch * X * N * N reals (N * (N+2) in place) */
    int64_t complex_bytes; /* batch * X * N * K complex (= send buffer)    */
    int64_t pencil_bytes;  /* batch * N * (N/p) * K complex, x-pencil      */
    int64_t chunk_bytes;   /* one all-to-all chunk: X * (N/p) * K complex  */
    /* Pencil plans (gfft_pencil_plan_create) reuse the fields above as:
     * slab_x = X = N/pr, ranks = pr * pc, real_bytes = batch * X * Y * N
     * reals, complex_bytes = batch * X * Y * K complex (first-exchange
     * order), pencil_bytes = batch * pc * X * Y * w complex (the y- and
     * x-pencils and the pr > pc send order), chunk_bytes = X * Y * w
     * complex (one first-exchange block per source rank, per grid; a
     * second-exchange block is pencil_bytes / (batch pr)).  Slab plans
     * report grid_r = p,
     * grid_c = 1, col = 0, y_local = N, kz_width = K. */
    int64_t grid_r;        /* pr: process-grid rows (x is cut pr ways)     */
    int64_t grid_c;        /* pc: process-grid columns (y, then kz)        */
    int64_t col;           /* this rank's column c, 0 <= c < pc            */
    int64_t y_local;       /* Y = N/pc local y extent of the real pencil   */
    int64_t kz_width;      /* w: kz bins this rank holds after exchange 1  */
} gfft_plan_sizes;

/*
 * Create a plan for one GPU's share of an N^3 real grid.
 *   n      : grid edge, a power of two with 16 <= n <= 4096 (the paper runs
 *            1024^3-4096^3; all sizes it uses are powers of two, section 2).
 *   dtype  : GFFT_F64 or GFFT_F32, the type of the data and the arithmetic.
 *   slab_x : local x-planes X; must divide n.  X == n is the full grid on
 *            one GPU (p = 1); X < n is rank r's slab of p = n/X ranks
 *            (section 2, slab decomposition).
 *   batch  : >= 1 independent grids per exec call.
 *   flags  : bitwise OR of GFFT_FUSE_PACK or GFFT_INPLACE,
 *            GFFT_PACK_PAPER_ORDER, and at most one of GFFT_MFMA_BF16X2 /
 *            GFFT_MFMA_BF16X3 (or 0).
 * On success *out receives the plan.  The plan owns small device tables
 * (FP64-derived twiddle factors rounded once to the working precision) on
 * the device that is current at creation; exec, pack and pass calls must run
 * with that device current (and on a stream of it), and return
 * GFFT_E_INVALID_ARG, before any launch, when another device is current.
 */
gfft_status gfft_plan_create(gfft_plan **out, int64_t n, gfft_dtype dtype,
                             int64_t slab_x, int64_t batch, uint32_t flags);

/*
 * Create a plan for one GPU's share of a pencil-decomposed N^3 real grid
 * (section 2, pencil decomposition: p = pr x pc processors, each holding
 * (N/pr) x (N/pc) x N real values; up to N^2/2 processors here, so p may
 * exceed N, the slab limit).  Rank (r, c) owns x in [r X, (r+1) X) and y in
 * [c Y, (c+1) Y), X = N/pr, Y = N/pc, all z.  The forward transform is
 *   1. gfft_exec_z_r2c: rows [batch][X][Y][N] -> half-spectrum rows written
 *      straight in first-exchange order: chunk c' (for rank (r, c')) holds
 *      kz in [c' w0, (c'+1) w0), w0 = N/(2 pc), and the last chunk also the
 *      Nyquist bin kz = N/2; chunk c' is a [X][Y][w_c'] block and the chunks
 *      lie back to back (X Y K complex per grid).
 *   2. exchange 1 (caller, among the pc ranks of row r): rank (r, c)
 *      receives chunk c of every (r, c') into block c' of its y-pencil
 *      [pc][X][Y][w] (w = w_c): element (c', x_l, y_l, kz_l) is
 *      (x = r X + x_l, y = c' Y + y_l, kz = c w0 + kz_l).
 *   3. gfft_exec_y_c2c: in place along y on that y-pencil.
 *   4. exchange 2 (caller, among the pr ranks of column c).  pr <= pc: with
 *      g = pc/pr, blocks c' in [r' g, (r'+1) g) of the y-pencil -- one
 *      contiguous run of g X Y w values -- go to rank (r', c), which stores
 *      the run from rank (r, c) as block r of its x-pencil
 *      [pr][g][X][Y][w]: element (r, g_l, x_l, y_l, kz_l) is (x = r X + x_l,
 *      y = r' N/pr + g_l Y + y_l, kz = c w0 + kz_l).  pr > pc: with
 *      h = pr/pc, gfft_pack_slab_for_alltoall first splits every y-pencil
 *      block into h runs [X][N/pr][w] (send order [pc][h][X][N/pr][w]);
 *      run (c', s) goes to rank (c' h + s, c), which stores the run from
 *      rank (r, c) as block r of its x-pencil [pr][X][N/pr][w] = [N][N/pr][w]
 *      (x = r X + x_l, y = r' N/pr + y_l, kz = c w0 + kz_l).
 *   5. gfft_exec_x_c2c: in place along x on that x-pencil.
 * The inverse runs 5, 4, 3, 2, 1 backwards (gfft_exec_x_c2c and
 * gfft_exec_y_c2c with sign +1, the exchanges returning every block to its
 * sender, gfft_unpack_slab_from_alltoall undoing the pack when pr > pc,
 * gfft_exec_z_c2r reading the first-exchange order).  Each exchange is per
 * grid of the batch.
 *   grid_r, grid_c : pr, pc, powers of two with pr <= N, pc <= N/2.
 *   col            : this rank's c (it fixes w: w0, or w0 + 1 when
 *                    c = pc - 1).
 *   flags          : 0 or one of GFFT_MFMA_BF16X2 / GFFT_MFMA_BF16X3 (FP32,
 *                    N >= 32); the slab flags return GFFT_E_UNSUPPORTED.
 * gfft_exec_r2c / c2r and the adjoints return GFFT_E_UNSUPPORTED on pencil
 * plans (their local work is steps 1 and 5 apart), and so do the pack and
 * unpack when pr <= pc (no pack is needed); gfft_exec_z_r2c's
 * scale/weighted arguments give the adjoint's bin factors as for slabs.
 */
gfft_status gfft_pencil_plan_create(gfft_plan **out, int64_t n,
                                    gfft_dtype dtype, int64_t grid_r,
                                    int64_t grid_c, int64_t col,
                                    int64_t batch, uint32_t flags);

/* Free a plan and its tables (NULL is accepted).  The caller must ensure no
 * work using the plan is still queued. */
gfft_status gfft_plan_destroy(gfft_plan *plan);

/* Fill *sizes with the plan's dimensions and buffer sizes. */
gfft_status gfft_plan_query(const gfft_plan *plan, gfft_plan_sizes *sizes);

/*
 * Forward transform, section 2 forward equation, unnormalized.
 *   in_real  : [batch][X][N][N] reals, not modified.
 *   out_cplx : [batch][X][N][K] complex (send order with GFFT_FUSE_PACK).
 * Full grid (X == N): the whole 3D R2C, output F(kx, ky, kz) in natural
 * order.  Slab (X < N): section 3 step 1, the 2D R2C over (y, z) of each
 * local plane; steps 2-4 are the caller's exchange; step 5 is
 * gfft_exec_x_c2c on the received pencil.
 * in_real and out_cplx must not overlap (must be equal for GFFT_INPLACE).
 */
gfft_status gfft_exec_r2c(const gfft_plan *plan, const void *in_real,
                          void *out_cplx, void *stream);

/*
 * Inverse transform, section 2 inverse equation, unnormalized, times scale
 * (scale = 1/N^3 gives back the field after a forward pass; the paper's
 * separate normalization step, section 4).  For a half spectrum G that is
 * not Hermitian the result is
 *   f(j) = scale * sum_{k in half} w(kz) Re(G(k) exp(+2 pi i k.j / N)),
 *   w(0) = w(N/2) = 1, w = 2 otherwise,
 * i.e. the inverse DFT of G's Hermitian extension.
 *   in_cplx  : [batch][X][N][K] complex (send order with GFFT_FUSE_PACK).
 *              CLOBBERED: the y (and x) passes run in place on it.
 *   out_real : [batch][X][N][N] reals.  Must not overlap in_cplx (must be
 *              equal to it for GFFT_INPLACE, rows then padded to N + 2).
 * Slab plans run the inverse of step 1 only (see gfft_exec_r2c).
 */
gfft_status gfft_exec_c2r(const gfft_plan *plan, void *in_cplx,
                          void *out_real, double scale, void *stream);

/*
 * Adjoint of the forward transform under the real inner products
 * <F,G> = sum_{k in half} Re(conj(F) G) and <f,h> = sum_j f h:
 *   out_real = scale * R2C^T(G) = scale * C2R(G / w).
 * Same layouts, aliasing rules and clobbering as gfft_exec_c2r.  This is
 * the gradient of a real loss through the forward transform when G holds
 * dL/dRe F + i dL/dIm F.
 */
gfft_status gfft_exec_r2c_adjoint(const gfft_plan *plan, void *in_cplx,
                                  void *out_real, double scale, void *stream);

/*
 * Adjoint of the inverse transform: out_cplx = scale * w * R2C(h), the
 * gradient of a real loss through gfft_exec_c2r(..., scale, ...) when h
 * holds dL/df.  Same layouts and aliasing rules as gfft_exec_r2c.
 */
gfft_status gfft_exec_c2r_adjoint(const gfft_plan *plan, const void *in_real,
                                  void *out_cplx, double scale, void *stream);

/*
 * Section 3 steps 2-3 as one permutation (standalone form of what
 * GFFT_FUSE_PACK folds into the z pass): from a slab's natural half
 * spectrum S[X][N][K], write p contiguous chunks
 *   send[j][x_l][y_l][kz] = S[x_l][j*(N/p) + y_l][kz],   j = 0..p-1,
 * chunk j destined for rank j.  Inside a chunk the order is [x_l][y_l][kz]:
 * after the exchange, rank r's received chunks read as one [N][N/p][K]
 * pencil (x slowest), so the paper's chunk transpose (step 4) is not needed.
 * A pure copy: bit-exact.  Per batch entry; buffers of plan complex_bytes;
 * they must not overlap.
 */
gfft_status gfft_pack_slab_for_alltoall(const gfft_plan *plan,
                                        const void *slab_cplx,
                                        void *send_blocks, void *stream);

/* Inverse permutation of gfft_pack_slab_for_alltoall (for the inverse
 * transform's return trip).  Bit-exact; buffers must not overlap. */
gfft_status gfft_unpack_slab_from_alltoall(const gfft_plan *plan,
                                           const void *recv_blocks,
                                           void *slab_cplx, void *stream);

/*
 * Section 3 step 5: in-place strided batched 1D complex FFT along x of the
 * pencil [batch][N][N/p][K] (x slowest, stride (N/p)*K), sign -1 forward,
 * +1 inverse, unnormalized.  For a full-grid plan (p = 1) this is the x
 * pass of the 3D transform on [N][N][K].
 */
gfft_status gfft_exec_x_c2c(const gfft_plan *plan, void *pencil, int sign,
                            void *stream);

/*
 * The individual passes, for timing each one and for composing the slab
 * pipeline by hand.  `data`/`in`/`out` follow the layouts above; the y pass
 * works in place on [batch][X][N][K] (send order with GFFT_FUSE_PACK).
 *   gfft_exec_z_r2c : rows of N reals -> rows of K complex (send-order
 *                     rows with GFFT_FUSE_PACK), times scale on every bin
 *                     and an extra factor 2 on 0 < kz < N/2 when weighted
 *                     is nonzero (the w of the adjoint).
 *   gfft_exec_y_c2c : 1D FFT along y, sign -1 or +1.
 *   gfft_exec_z_c2r : rows of K complex -> N reals with Im of kz = 0 and
 *                     kz = N/2 discarded, times scale, bins 0 < kz < N/2
 *                     halved first when weighted is nonzero.
 */
gfft_status gfft_exec_z_r2c(const gfft_plan *plan, const void *in_real,
                            void *out_cplx, double scale, int weighted,
                            void *stream);
gfft_status gfft_exec_y_c2c(const gfft_plan *plan, void *data, int sign,
                            void *stream);
gfft_status gfft_exec_z_c2r(const gfft_plan *plan, const void *in_cplx,
                            void *out_real, double scale, int weighted,
                            void *stream);

/*
 * Plain device-to-device copy of `bytes` bytes (a multiple of 16; both
 * pointers 16-byte aligned, in memory the current device can access; the
 * buffers must not overlap), one 16-byte element per work-item, enqueued on
 * `stream` (a stream of the current device).  Not a step of
 * the transform: it is the reference rate for contiguous HBM traffic
 * against which the passes' bandwidth is judged (a pass that reads and
 * writes B bytes cannot beat a copy of B/2 bytes).  A zero-byte copy does
 * nothing.
 */
gfft_status gfft_device_copy(void *dst, const void *src, int64_t bytes,
                             void *stream);

/*
 * Access-pattern yardstick of a strided pass (not a step of the transform):
 * reads and writes every element that gfft_exec_y_c2c (axis 0) or
 * gfft_exec_x_c2c (axis 1) would, in place, with that pass's tile shape,
 * workgroup order and memory hints, but runs no transform: each element is
 * replaced by its complex conjugate.  Its rate is the ceiling of the pass's
 * memory access pattern (the pass without its arithmetic and exchanges).
 *   data : the buffer gfft_exec_y_c2c / gfft_exec_x_c2c takes on this plan
 *          (same layout, size, alignment and device rules).
 * Errors: GFFT_E_INVALID_ARG for a NULL plan or pointer, an axis other than
 * 0 or 1, or a current device other than the plan's; GFFT_E_ALIGN;
 * GFFT_E_HIP for a launch failure.
 */
gfft_status gfft_exec_pass_copy(const gfft_plan *plan, int axis, void *data,
                                void *stream);

/* Static description of a status code (never NULL). */
const char *gfft_status_string(gfft_status status);

/* Library version as major*10000 + minor*100 + patch. */
int gfft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GFFT_H */
