// Kernel launchers of the slab 3D real FFT (host-callable, C++ linkage).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gfft {

// Maps a natural row index r of the [batch][X][N] row space (one row = one
// z-line) to the row it occupies in a half-spectrum buffer: the natural row
// when lg_y == lg_n, or the all-to-all send order [p][X][N/p] of the slab's
// chunks (chunk j = y / (N/p)) otherwise.  All extents are powers of two.
// rs is the distance between real rows, in reals: N, or N + 2 for the
// padded rows of an in-place transform (a real row and its K complex bins
// then share the same bytes).
// paper != 0 selects the chunk order of the paper's local xy transpose,
// [p][N/p][X] = the slab transposed to [N][X] (row (x_l, y) at y X + x_l).
// pencil != 0 selects the first-exchange order of a pencil plan instead: the
// K bins of row r = item * 2^lg_rows + r_l are cut into pc = pc_last + 1
// chunks, chunk c holding kz in [c w, (c+1) w) with w = 2^lg_w = N/(2 pc)
// and the last chunk also kz = N/2; chunk c is a [2^lg_rows][w_c] block at
// item * 2^lg_rows * K + c * 2^lg_rows * w.
struct row_map {
    int lg_n, lg_x, lg_y;
    int64_t rs;
    int paper;
    int pencil = 0, lg_rows = 0, lg_w = 0, pc_last = 0;
};

// Address of element (b, n, m) of a batch of strided lines:
//   (b >> lg_bx) * b_hi + (b & (2^lg_bx - 1)) * b_lo
//   + (n >> lg_y) * s_hi + (n & (2^lg_y - 1)) * s_lo + m
// which covers the y lines of a natural or send-ordered slab and the x
// lines of a pencil.
struct line_map {
    int64_t b_hi, b_lo, s_hi, s_lo;
    int lg_bx, lg_y;
};

// All launchers return hipSuccess or the launch error.
// tw: device table of W_N^m = exp(-2 pi i m / N), m = 0..N-1, of type T.
hipError_t launch_z_r2c(bool f64, int n, const void* in, void* out, const void* tw,
                        int64_t rows, row_map map, double mul_edge, double mul_int,
                        hipStream_t s);
hipError_t launch_z_c2r(bool f64, int n, const void* in, void* out, const void* tw,
                        int64_t rows, row_map map, double mul_edge, double mul_int,
                        hipStream_t s);
// axis 0: y lines (short stride); axis 1: x lines (long stride).  Picks the
// tile shape measured best for that stride.  mfma_terms 2 or 3 (FP32, N >= 32
// only) runs the first radix-16 stage on the matrix cores with that many
// BF16 terms per operand; 0 keeps every stage on the vector ALUs; -1 runs
// no transform but the vector pass's loads and stores, storing each element's
// conjugate (sign ignored).
hipError_t launch_strided(bool f64, int n, int axis, int mfma_terms, int sign, void* data,
                          const void* tw, int64_t m_cols, int64_t n_b, line_map lm,
                          hipStream_t s);
// Copy `chunks` runs of `len` complex values: run c = (bb, j, xl) goes from
// natural offset bb*X*N*K + (xl*N + j*Y)*K to send offset
// bb*X*N*K + (j*X + xl)*Y*K (to_send = true) or back (to_send = false).
hipError_t launch_pack(bool f64, const void* src, void* dst, int64_t chunks,
                       int lg_x, int lg_p, int64_t n, int64_t y, int64_t k,
                       bool to_send, hipStream_t s);
// Copy `rows` rows of k complex values between the natural order and the
// order `map` describes (natural row r <-> map_row(r)), to_send choosing the
// direction.  Used for the paper's chunk order, whose rows interleave.
hipError_t launch_pack_rows(bool f64, const void* src, void* dst, int64_t rows, int64_t k,
                            row_map map, bool to_send, hipStream_t s);

// Step 1 (z R2C and y C2C of every x-plane) in one pass, or its inverse
// (y C2C, then z C2R), one plane per workgroup: FP32, N = 64 and 128 both
// ways, N = 256 forward only (plane_supported).  Rows of the half spectrum
// follow `map` as in the z passes; the bin multipliers are those of the z
// passes.  `in` and `out` may be the same buffer (in-place plans): each
// plane is read whole before any of it is written.
bool plane_supported(bool f64, int n, bool forward);
hipError_t launch_plane(bool f64, bool forward, int n, const void* in, void* out, const void* tw,
                        int64_t planes, row_map map, double mul_edge, double mul_int,
                        hipStream_t s);

// Copy n16 16-byte elements from src to dst (one per work-item).
hipError_t launch_copy16(const void* src, void* dst, int64_t n16, hipStream_t s);

}  // namespace gfft
