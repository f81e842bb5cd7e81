// HIP kernels of the slab 3D real FFT for gfx950 (MI355X).
//
// Three pass kinds cover the whole path (section 3 steps 1 and 5 and their
// inverse; steps 2-4 are row permutations folded into addressing):
//   z pass  : contiguous rows.  A row of N reals is read as N/2 complex
//             values z[n] = x[2n] + i x[2n+1], transformed with an N/2-point
//             complex FFT, and split into the K = N/2+1 bins of the real
//             transform (and the reverse for C2R).
//   y/x pass: strided lines.  A workgroup owns TC adjacent columns of a
//             batch of lines; lanes of consecutive columns read consecutive
//             addresses, so every load and store is a contiguous run of
//             TC complex values per line position.
//   pack    : the send-order permutation as a plain copy of contiguous runs.
// Pencil plans (section 2, pencil decomposition) reuse the same passes: the
// z pass scatters each row's bins to the first exchange's chunks, and the
// y/x passes address the received pencils through their line maps.
// Memory bound: each pass reads and writes its array once.
#include "cx.h"
#include "engine.h"
#include "kernels.h"
#include "mfma_dft16.h"

namespace gfft {

constexpr int kThreads = 256;

constexpr int ilog2_c(int v) { return v <= 1 ? 0 : 1 + ilog2_c(v / 2); }

// Largest radix per FFT stage.  The FP32 vector kernels take radix-32
// stages, one LDS exchange fewer for 512- and 1024-point transforms (FP32 is
// bound by instruction issue); FP64 and the matrix-core stage keep radix 16.
template <typename T, int MF = 0>
constexpr int radix_cap() { return sizeof(T) == 4 && MF == 0 ? 32 : 16; }

// A workgroup-uniform value in scalar registers that the optimiser cannot
// see through: expressions of it are formed where they are used.
__device__ __forceinline__ int opaque_uniform(int v) {
    int r = __builtin_amdgcn_readfirstlane(v);
    asm volatile("" : "+s"(r));
    return r;
}
__device__ __forceinline__ int64_t opaque_uniform(int64_t v) {
    const uint64_t u = uint64_t(v);
    const uint32_t lo = uint32_t(opaque_uniform(int(uint32_t(u)))),
                   hi = uint32_t(opaque_uniform(int(uint32_t(u >> 32))));
    return int64_t((uint64_t(hi) << 32) | lo);
}

__device__ __forceinline__ int64_t map_row(int64_t r, row_map m) {
    const int64_t bx = r >> m.lg_n;
    const int64_t y = r & ((int64_t(1) << m.lg_n) - 1);
    const int64_t b = bx >> m.lg_x;
    const int64_t xl = bx & ((int64_t(1) << m.lg_x) - 1);
    if (m.paper) return (b << (m.lg_x + m.lg_n)) + (y << m.lg_x) + xl;
    const int64_t j = y >> m.lg_y;
    const int64_t yl = y & ((int64_t(1) << m.lg_y) - 1);
    return (b << (m.lg_x + m.lg_n)) + ((((j << m.lg_x) + xl)) << m.lg_y) + yl;
}

// Offset (in complex values) of bin k of row r in a pencil plan's
// first-exchange order (row_map::pencil).
__device__ __forceinline__ int64_t pencil_bin(int64_t r, int k, int K, const row_map& m) {
    const int64_t item = r >> m.lg_rows;
    const int64_t rl = r & ((int64_t(1) << m.lg_rows) - 1);
    const int c = (k >> m.lg_w) < m.pc_last ? (k >> m.lg_w) : m.pc_last;
    const int64_t wc = (int64_t(1) << m.lg_w) + (c == m.pc_last ? 1 : 0);
    return ((item * K + (int64_t(c) << m.lg_w)) << m.lg_rows) + rl * wc + (k - (c << m.lg_w));
}

// Consecutive workgroup ids are dealt round-robin to the 8 XCDs, each with
// its own L2.  Remap so that XCD x works through one contiguous range of
// tiles: neighbouring tiles share cache lines at their edges.
__device__ __forceinline__ int64_t xcd_tile(int64_t g, int64_t G) {
    constexpr int kXcd = 8;
    const int64_t per = G / kXcd;
    if (g >= per * kXcd) return g;
    return (g % kXcd) * per + g / kXcd;
}

template <int M, int EMAX = 16, int THREADS = kThreads>
struct zshape {
    static constexpr int E = M < EMAX ? M : EMAX;  // elements per thread
    static constexpr int TPT = M / E;              // threads per row
    static constexpr int NT = THREADS > TPT ? THREADS : TPT;
    static constexpr int RPB = NT / TPT;           // rows per workgroup
};

// Workgroup shape of the z passes, chosen by measurement (2^18 and 2^20
// rows): FP64 R2C 8 elements per thread in 256-thread workgroups up to
// N = 512, 16 per thread in 128-thread ones for N = 1024 and 2048 (7-8%
// faster there), 32 per thread for N = 4096; FP64 C2R 16 per thread in
// 64-thread workgroups; FP32 32 per thread, in 256-thread workgroups for the
// R2C from N = 1024 up (4-10% faster with the radix-32 stages) and 64-thread
// ones otherwise, except at N = 256 and 512: 16 per thread in 256-thread
// workgroups (the C2R of N = 512 in 128-thread ones), 5-13% faster there.
// Workgroups are dealt to XCDs in contiguous ranges by the C2R at every N
// (3-5%) and by the R2C from N = 1024 up (2-3%) and at the FP32 N = 256 and
// 512 shapes.  The C2R also stores its line-aligned real rows
// non-temporally (they are not read again soon); the R2C's complex rows are
// not line-aligned and gain nothing from it.
template <typename T, bool FWD, int N>
struct zcfg {
    static constexpr bool F64 = sizeof(T) == 8;
    static constexpr bool MID32 = !F64 && (N == 256 || N == 512);
    static constexpr int EMAX =
        F64 ? (FWD ? (N >= 4096 ? 32 : N >= 1024 ? 16 : 8) : 16) : (MID32 ? 16 : 32);
    static constexpr int THREADS =
        F64 ? (FWD ? (N >= 1024 ? 128 : 256) : 64)
            : MID32 ? (FWD || N == 256 ? 256 : 128) : (FWD && N >= 1024 ? 256 : 64);
    static constexpr bool REMAP = !FWD || N >= 1024 || MID32;
    static constexpr bool NTS = !FWD;
};

// ---------------------------------------------------------------- z R2C
// ALIAS: `in` and `out` are the same buffer (in-place plans).  Each row is
// read completely before the first barrier and written after the last one,
// so a row is never overwritten before all of it has been loaded.
template <typename T, int N, int EMAX, int THREADS, bool REMAP, bool NTS, bool ALIAS,
          bool PENCIL = false>
__device__ __forceinline__ void z_r2c_body(
    const T* in, cx<T>* out, const cx<T>* __restrict__ tw,
    int64_t rows, row_map map, T mul_edge, T mul_int) {
    constexpr int M = N / 2, K = M + 1;
    using Z = zshape<M, EMAX, THREADS>;
    constexpr int E = Z::E, TPT = Z::TPT, RPB = Z::RPB;
    constexpr int RM = radix_cap<T>();
    constexpr int PS = first_radix_shift<E, RM>::value, MP = padded_len<M, PS>::value;
    __shared__ cx<T> lds[RPB * MP];

    const int rl = threadIdx.x / TPT;
    const int t = threadIdx.x % TPT;
    const int64_t blk = REMAP ? xcd_tile(blockIdx.x, gridDim.x) : int64_t(blockIdx.x);
    const int64_t row = blk * RPB + rl;
    const bool valid = row < rows;

    // Rows past the end (last workgroup) load the last row and discard it.
    const cx<T>* src = reinterpret_cast<const cx<T>*>(in + (valid ? row : rows - 1) * map.rs);
    cx<T> a[E];
#pragma unroll
    for (int m = 0; m < E; ++m) a[m] = src[t + m * TPT];

    const idx_rows<PS> ix{rl * MP};
    fft_regs<T, M, E, -1, RM>(a, t, tw, 2, xch_full<T, idx_rows<PS>>{lds, ix});

    // Split Z = FFT_M(z) into the real transform:
    //   X[k] = (Z[k] + conj Z[M-k])/2 - (i/2) W_N^k (Z[k] - conj Z[M-k]),
    //   X[M] = Re Z[0] - Im Z[0].
#pragma unroll
    for (int m = 0; m < E; ++m) lds[ix.at(xgeom<M, E, 1, 1>::template in_pad<PS>(t, m))] = a[m];
    __syncthreads();
    if (!valid) return;
    // With ALIAS, all bins are formed in registers before the first store:
    // stores through a pointer that may alias `in` would otherwise keep the
    // twiddle loads from being issued early.
    const cx<T> x_m{(a[0].x - a[0].y) * mul_edge, T(0)};
    cx<T>* dst = out + (PENCIL ? 0 : map_row(row, map) * K);
    auto put = [&](int k, cx<T> v) {
        if constexpr (PENCIL) {
            out[pencil_bin(row, k, K, map)] = v;
        } else if constexpr (NTS) {
            __builtin_nontemporal_store(v.x, &dst[k].x);
            __builtin_nontemporal_store(v.y, &dst[k].y);
        } else {
            dst[k] = v;
        }
    };
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = t + m * TPT;
        const cx<T> zk = a[m];
        const cx<T> zc = conjg(lds[ix((M - k) & (M - 1))]);
        const cx<T> A = scal(zk + zc, T(0.5));
        const cx<T> B = scal(zk - zc, T(0.5));
        const cx<T> wb = cmul(tw[k], B);
        const T f = k == 0 ? mul_edge : mul_int;
        const cx<T> v{(A.x + wb.y) * f, (A.y - wb.x) * f};
        if constexpr (ALIAS) a[m] = v;
        else put(k, v);
    }
    if constexpr (ALIAS) {
#pragma unroll
        for (int m = 0; m < E; ++m) put(t + m * TPT, a[m]);
    }
    if (t == 0) put(M, x_m);
}

template <typename T, int N, int EMAX, int THREADS, bool REMAP, bool NTS>
__global__ __launch_bounds__((zshape<N / 2, EMAX, THREADS>::NT)) void k_z_r2c(
    const T* __restrict__ in, cx<T>* __restrict__ out, const cx<T>* __restrict__ tw,
    int64_t rows, row_map map, T mul_edge, T mul_int) {
    z_r2c_body<T, N, EMAX, THREADS, REMAP, NTS, false>(in, out, tw, rows, map, mul_edge, mul_int);
}

template <typename T, int N, int EMAX, int THREADS, bool REMAP, bool NTS>
__global__ __launch_bounds__((zshape<N / 2, EMAX, THREADS>::NT)) void k_z_r2c_inplace(
    const T* in, cx<T>* out, const cx<T>* __restrict__ tw,
    int64_t rows, row_map map, T mul_edge, T mul_int) {
    z_r2c_body<T, N, EMAX, THREADS, REMAP, NTS, true>(in, out, tw, rows, map, mul_edge, mul_int);
}

// Pencil plans: bins scattered to the first exchange's chunks.
template <typename T, int N, int EMAX, int THREADS, bool REMAP>
__global__ __launch_bounds__((zshape<N / 2, EMAX, THREADS>::NT)) void k_z_r2c_pencil(
    const T* __restrict__ in, cx<T>* __restrict__ out, const cx<T>* __restrict__ tw,
    int64_t rows, row_map map, T mul_edge, T mul_int) {
    z_r2c_body<T, N, EMAX, THREADS, REMAP, false, false, true>(in, out, tw, rows, map, mul_edge,
                                                               mul_int);
}

// ---------------------------------------------------------------- z C2R
template <typename T, int N, int EMAX, int THREADS, bool REMAP, bool NTS, bool PENCIL = false>
__device__ __forceinline__ void z_c2r_body(
    const cx<T>* in, T* out, const cx<T>* __restrict__ tw,
    int64_t rows, row_map map, T mul_edge, T mul_int) {
    constexpr int M = N / 2, K = M + 1;
    using Z = zshape<M, EMAX, THREADS>;
    constexpr int E = Z::E, TPT = Z::TPT, RPB = Z::RPB;
    constexpr int RM = radix_cap<T>();
    constexpr int PS = first_radix_shift<E, RM>::value, MP = padded_len<M, PS>::value;
    __shared__ cx<T> lds[RPB * MP];

    const int rl = threadIdx.x / TPT;
    const int t = threadIdx.x % TPT;
    const int64_t blk = REMAP ? xcd_tile(blockIdx.x, gridDim.x) : int64_t(blockIdx.x);
    const int64_t row = blk * RPB + rl;
    const bool valid = row < rows;
    const idx_rows<PS> ix{rl * MP};

    // Load G[0..M-1] (registers and LDS) and G[M] (thread t = 0), dropping
    // the imaginary parts of kz = 0 and kz = N/2 and applying the bin
    // multipliers (scale, and 1/w for the adjoint).
    // Rows past the end (last workgroup) load the last row and discard it.
    cx<T> g[E];
    cx<T> g_m;
    const int64_t lrow = valid ? row : rows - 1;
    if constexpr (PENCIL) {
#pragma unroll
        for (int m = 0; m < E; ++m) g[m] = in[pencil_bin(lrow, t + m * TPT, K, map)];
        g_m = t == 0 ? in[pencil_bin(lrow, M, K, map)] : cx<T>{T(0), T(0)};
    } else {
        const cx<T>* src = in + map_row(lrow, map) * K;
#pragma unroll
        for (int m = 0; m < E; ++m) g[m] = src[t + m * TPT];
        g_m = t == 0 ? src[M] : cx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = t + m * TPT;
        if (k == 0) g[m] = cx<T>{g[m].x * mul_edge, T(0)};
        else g[m] = scal(g[m], mul_int);
        lds[ix.at(xgeom<M, E, 1, 1>::template in_pad<PS>(t, m))] = g[m];
    }
    g_m = cx<T>{g_m.x * mul_edge, T(0)};
    __syncthreads();

    // Z'[k] = (G[k] + conj G[M-k]) + i conj(W_N^k) (G[k] - conj G[M-k]);
    // its inverse M-point FFT interleaves the even and odd outputs.
    cx<T> a[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = t + m * TPT;
        const cx<T> gc = conjg(k == 0 ? g_m : lds[ix(M - k)]);
        const cx<T> s = g[m] + gc;
        const cx<T> d = cmulc(g[m] - gc, tw[k]);
        a[m] = cx<T>{s.x - d.y, s.y + d.x};
    }
    __syncthreads();
    fft_regs<T, M, E, +1, RM>(a, t, tw, 2, xch_full<T, idx_rows<PS>>{lds, ix});
    if (!valid) return;
    cx<T>* dst = reinterpret_cast<cx<T>*>(out + row * map.rs);
#pragma unroll
    for (int m = 0; m < E; ++m) {
        if constexpr (NTS) {
            __builtin_nontemporal_store(a[m].x, &dst[t + m * TPT].x);
            __builtin_nontemporal_store(a[m].y, &dst[t + m * TPT].y);
        } else {
            dst[t + m * TPT] = a[m];
        }
    }
}

template <typename T, int N, int EMAX, int THREADS, bool REMAP, bool NTS>
__global__ __launch_bounds__((zshape<N / 2, EMAX, THREADS>::NT)) void k_z_c2r(
    const cx<T>* __restrict__ in, T* __restrict__ out, const cx<T>* __restrict__ tw,
    int64_t rows, row_map map, T mul_edge, T mul_int) {
    z_c2r_body<T, N, EMAX, THREADS, REMAP, NTS>(in, out, tw, rows, map, mul_edge, mul_int);
}

// In place: every load of a row precedes the barrier after the LDS fill, and
// every store follows the last barrier of the FFT.
template <typename T, int N, int EMAX, int THREADS, bool REMAP, bool NTS>
__global__ __launch_bounds__((zshape<N / 2, EMAX, THREADS>::NT)) void k_z_c2r_inplace(
    const cx<T>* in, T* out, const cx<T>* __restrict__ tw,
    int64_t rows, row_map map, T mul_edge, T mul_int) {
    z_c2r_body<T, N, EMAX, THREADS, REMAP, NTS>(in, out, tw, rows, map, mul_edge, mul_int);
}

// Pencil plans: bins gathered from the first exchange's chunks.
template <typename T, int N, int EMAX, int THREADS, bool REMAP, bool NTS>
__global__ __launch_bounds__((zshape<N / 2, EMAX, THREADS>::NT)) void k_z_c2r_pencil(
    const cx<T>* __restrict__ in, T* __restrict__ out, const cx<T>* __restrict__ tw,
    int64_t rows, row_map map, T mul_edge, T mul_int) {
    z_c2r_body<T, N, EMAX, THREADS, REMAP, NTS, true>(in, out, tw, rows, map, mul_edge, mul_int);
}

// ---------------------------------------------------------------- plane 2D R2C / C2R
// Step 1 of the method (the 2D R2C over (y, z) of one x-plane) in one kernel
// when a plane fits on a CU: FP32, N = 64, 128, 256 (a 256 x 256 plane is
// 256 KiB of reals and 264 KiB of half spectrum; the register file holds it),
// and the inverse for N = 64 and 128 (plane_supported says where each runs).
// One workgroup per plane, NT = N M / 32 threads, 32 complex values per
// thread in both phases:
//   z phase: thread (r, t), r < N rows, t < TZ = M/32, holds z[t + TZ m] of
//            row r (z[n] = x[2n] + i x[2n+1]); M-point FFT;
//   y phase: thread (s, c), c < M columns, s < TY = N/32, holds column c at
//            rows s + TY m; N-point FFT.
// Between the phases the plane moves through LDS, real parts then imaginary
// parts.  The forward's real split (bin k from Z[k] and Z[M-k]) is formed
// by the column threads as they read the transposed plane, column c taking
// columns c and M - c from LDS; the inverse forms its pre-process the same
// way after the transpose back, through a mirror exchange of half the rows
// at a time.  The z half spectrum has M + 1 columns; kz = 0 and kz = M are real
// for a real row, so they travel together as one complex column
// P = X[.][0] + i X[.][M] (two real transforms for one complex one) and are
// separated after the y FFT: X0 = (P + conj P(-ky)) / 2, XM = (P - conj
// P(-ky)) / 2i.  The inverse packs the Hermitian parts of the kz = 0 and
// kz = M columns the same way (the C2R keeps only the real part of those
// columns after the y inverse, which is the inverse of their Hermitian
// parts).  Every load of a plane precedes the first barrier and every store
// follows the last, so the plane may be transformed in place.
template <int N>
struct plane_shape {
    static constexpr int M = N / 2, K = M + 1;
    static constexpr int E = 32;
    static constexpr int TZ = M / E, TY = N / E;
    static constexpr int NT = N * TZ;  // = M * TY
    static constexpr int PS = 5;       // first radix 32: one pad per 32 positions
    static constexpr int MP = M + (M >> PS);
    static constexpr int NP = N + (N >> PS);
    static constexpr int LD = M + 1;   // odd row stride of the transpose buffer
    static constexpr int A = N * MP, B = NP * M, C = N * LD, D = (N / 2) * MP * 2;
    static constexpr int AB = A > B ? A : B, CD = C > D ? C : D;
    static constexpr int LDS = AB > CD ? AB : CD;  // floats
    static_assert(TZ >= 1 && TY >= 1 && N * TZ == M * TY, "plane shape");
};

// The z phase's mirror exchange: every thread replaces v[m] (bin
// k = t + TZ m of row r) by f(m, v[m], v_r[(M - k) mod M]), the mirror value
// read back through LDS as a whole complex value; half of the rows at a time.
template <int N, class F>
__device__ __forceinline__ void plane_mirror(float* lds, int r, int t, cx<float> (&v)[32],
                                             F&& f) {
    using P = plane_shape<N>;
    cx<float>* buf = reinterpret_cast<cx<float>*>(lds);
    const int rl = r & (N / 2 - 1);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const bool mine = (r >= N / 2) == (half != 0);
        if (mine) {
#pragma unroll
            for (int m = 0; m < 32; ++m) buf[rl * P::MP + t + P::TZ * m] = v[m];
        }
        __syncthreads();
        if (mine) {
#pragma unroll
            for (int m = 0; m < 32; ++m)
                v[m] = f(m, v[m], buf[rl * P::MP + ((P::M - (t + P::TZ * m)) & (P::M - 1))]);
        }
        __syncthreads();
    }
}

template <int N>
__global__ __launch_bounds__(plane_shape<N>::NT) void k_plane_r2c(
    const float* in, cx<float>* out, const cx<float>* __restrict__ tw, int64_t planes,
    row_map map, float mul_edge, float mul_int) {
    using P = plane_shape<N>;
    constexpr int M = P::M, K = P::K, TZ = P::TZ, TY = P::TY;
    __shared__ float lds[P::LDS];
    const int64_t plane = blockIdx.x;
    const int tid = threadIdx.x;
    const int r = tid / TZ, t = tid % TZ;  // z phase
    const int c = tid % M, s = tid / M;    // y phase

    // z phase: row r of the plane, read as M complex values
    cx<float> a[32];
    const cx<float>* src = reinterpret_cast<const cx<float>*>(in + (plane * N + r) * map.rs);
#pragma unroll
    for (int m = 0; m < 32; ++m) a[m] = src[t + TZ * m];
    fft_regs<float, M, 32, -1, 32>(a, t, tw, 2,
                                   xch_split<float, idx_rows<P::PS>>{lds, idx_rows<P::PS>{r * P::MP}});

    // rows -> columns, real then imaginary parts, with the real split folded
    // in: column thread c reads Z[y][c] and Z[y][M-c] and forms
    //   X[c] = (Z[c] + conj Z[M-c])/2 - (i/2) W_N^c (Z[c] - conj Z[M-c])
    // as a part from the real parts and a part from the imaginary parts
    // (bin multipliers applied); kz = 0 and kz = M (both real, X[M] =
    // Re Z[0] - Im Z[0]) travel as one complex column c = 0.
    const int cm = (M - c) & (M - 1);
    const cx<float> w = tw[c];
    const float f = c == 0 ? mul_edge : mul_int;
    cx<float> b[32];
#pragma unroll
    for (int m = 0; m < 32; ++m) lds[r * P::LD + t + TZ * m] = a[m].x;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 32; ++m) {
        const float zr = lds[(s + TY * m) * P::LD + c], mr = lds[(s + TY * m) * P::LD + cm];
        const float hd = 0.5f * (zr - mr);
        b[m] = cx<float>{0.5f * (zr + mr) + w.y * hd, -w.x * hd};
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 32; ++m) lds[r * P::LD + t + TZ * m] = a[m].y;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 32; ++m) {
        const float zi = lds[(s + TY * m) * P::LD + c], mi = lds[(s + TY * m) * P::LD + cm];
        const float hs = 0.5f * (zi + mi);
        const float vx = b[m].x + w.x * hs;
        // c = 0: b[m].x holds Re Z[0], the imaginary part carries X[M]
        const float vy = c == 0 ? b[m].x - zi : b[m].y + 0.5f * (zi - mi) + w.y * hs;
        b[m] = cx<float>{vx * f, vy * f};
    }
    __syncthreads();

    // y phase: column c, N-point FFT
    fft_regs<float, N, 32, -1, 32>(b, s, tw, 1,
                                   xch_split<float, idx_cols<M, P::PS>>{lds, idx_cols<M, P::PS>{c}});

    // separate the packed column: thread (s, 0) needs P(-ky) from (s', 0)
    cx<float>* col0 = reinterpret_cast<cx<float>*>(lds);
    if (c == 0) {
#pragma unroll
        for (int m = 0; m < 32; ++m) col0[s + TY * m] = b[m];
    }
    __syncthreads();
    // store rows of the half spectrum: wave lanes are consecutive columns
#pragma unroll
    for (int m = 0; m < 32; ++m) {
        const int ky = s + TY * m;
        cx<float>* dst = out + map_row(plane * N + ky, map) * K;
        if (c == 0) {
            const cx<float> pc = conjg(col0[(N - ky) & (N - 1)]);
            const cx<float> sum = b[m] + pc, dif = b[m] - pc;
            dst[0] = cx<float>{0.5f * sum.x, 0.5f * sum.y};   // X[ky][0]
            dst[M] = cx<float>{0.5f * dif.y, -0.5f * dif.x};  // X[ky][M] = dif / 2i
        } else {
            dst[c] = b[m];
        }
    }
}

template <int N>
__global__ __launch_bounds__(plane_shape<N>::NT) void k_plane_c2r(
    const cx<float>* in, float* out, const cx<float>* __restrict__ tw, int64_t planes,
    row_map map, float mul_edge, float mul_int) {
    using P = plane_shape<N>;
    constexpr int M = P::M, K = P::K, TZ = P::TZ, TY = P::TY;
    __shared__ float lds[P::LDS];
    const int64_t plane = blockIdx.x;
    const int tid = threadIdx.x;
    const int r = tid / TZ, t = tid % TZ;
    const int c = tid % M, s = tid / M;

    // y phase input: column c of the half spectrum, bin multipliers applied;
    // column 0 carries the Hermitian parts of kz = 0 (real) and kz = M
    // (imaginary), formed through LDS
    cx<float> b[32];
    cx<float>* col0 = reinterpret_cast<cx<float>*>(lds);
#pragma unroll
    for (int m = 0; m < 32; ++m) {
        const int ky = s + TY * m;
        const cx<float>* row = in + map_row(plane * N + ky, map) * K;
        if (c == 0) {
            col0[ky] = scal(row[0], mul_edge);
            col0[N + ky] = scal(row[M], mul_edge);
        } else {
            b[m] = scal(row[c], mul_int);
        }
    }
    __syncthreads();
    if (c == 0) {
#pragma unroll
        for (int m = 0; m < 32; ++m) {
            const int ky = s + TY * m, kn = (N - ky) & (N - 1);
            const cx<float> h0 = scal(col0[ky] + conjg(col0[kn]), 0.5f);
            const cx<float> hm = scal(col0[N + ky] + conjg(col0[N + kn]), 0.5f);
            b[m] = cx<float>{h0.x - hm.y, h0.y + hm.x};  // h0 + i hm
        }
    }
    __syncthreads();
    fft_regs<float, N, 32, +1, 32>(b, s, tw, 1,
                                   xch_split<float, idx_cols<M, P::PS>>{lds, idx_cols<M, P::PS>{c}});

    // columns -> rows, real then imaginary parts; column 0's real part is
    // G[y][0] and its imaginary part G[y][M], both real bins of the z C2R
    cx<float> g[32];
#pragma unroll
    for (int m = 0; m < 32; ++m) lds[(s + TY * m) * P::LD + c] = b[m].x;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 32; ++m) g[m].x = lds[r * P::LD + t + TZ * m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 32; ++m) lds[(s + TY * m) * P::LD + c] = b[m].y;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 32; ++m) g[m].y = lds[r * P::LD + t + TZ * m];
    __syncthreads();
    // thread t = 0 of row r: g[0] = (G[0], G[M]) as read; split them
    const float g_m = g[0].y;
    if (t == 0) g[0].y = 0.f;

    // z C2R: Z'[k] = (G[k] + conj G[M-k]) + i conj(W_N^k) (G[k] - conj G[M-k]),
    // with G[M] = g_m for k = 0
    plane_mirror<N>(lds, r, t, g, [&](int m, cx<float> gk, cx<float> gmir) {
        const int k = t + TZ * m;
        const cx<float> gc = conjg(k == 0 ? cx<float>{g_m, 0.f} : gmir);
        const cx<float> sm = gk + gc;
        const cx<float> d = cmulc(gk - gc, tw[k]);
        return cx<float>{sm.x - d.y, sm.y + d.x};
    });
    fft_regs<float, M, 32, +1, 32>(g, t, tw, 2,
                                   xch_split<float, idx_rows<P::PS>>{lds, idx_rows<P::PS>{r * P::MP}});
    cx<float>* dst = reinterpret_cast<cx<float>*>(out + (plane * N + r) * map.rs);
#pragma unroll
    for (int m = 0; m < 32; ++m) dst[t + TZ * m] = g[m];
}

// ---------------------------------------------------------------- y / x C2C
// Tile shape of the strided pass: TC columns of length N per workgroup, E
// elements per thread (TPT = N/E threads per column), exchanges through LDS
// either as whole complex values or split into real and imaginary halves
// (half the LDS per tile, twice the barriers).  Chosen by measurement at
// 1024^3 (FP64: y 16 columns, 512 threads, 128 KiB; x 8 columns, 256
// threads, 64 KiB; FP32: 16 columns, 512 threads, 64 KiB, both axes):
//   AX = 0 (y lines, rows K apart) and any N >= 2048 get the wide budget,
//   AX = 1 (x lines, rows megabytes apart) keeps two tiles per CU in FP64.
// TC is at most 16 columns unless the lines are so short that 256 threads
// need more.
template <typename T, int N, int AX, bool MFMA = false>
struct sshape {
    static constexpr bool F64 = sizeof(T) == 8;
    static constexpr bool WIDE = AX == 0 || N >= 2048;
    // FP32 lines of N = 256 and x lines of N = 512: 32 columns (256-byte
    // runs), 4% faster than 16 (at N = 256 the x tile with 32 elements per
    // thread, the y tile with 16)
    static constexpr bool C32 = !F64 && !MFMA && (N == 256 || (N == 512 && AX == 1));
    static constexpr int E = MFMA ? 16 : (N >= 512 || (C32 && AX == 1)) ? 32 : 16;
    static constexpr int TPT = N / E;
    // FP32 y lines of N = 2048: two 8-column tiles per CU (9% faster than
    // one 16-column tile); FP64 y lines of N = 512: two 16-column tiles with
    // the split exchange (8% faster than one with whole values)
    static constexpr bool Y2048 = !F64 && !MFMA && AX == 0 && N == 2048;
    static constexpr bool Y512 = F64 && AX == 0 && N == 512;
    static constexpr bool BIG32 = N >= 2048 && !Y2048;
    static constexpr int MAXT = F64 ? (WIDE ? 512 : 256) : (BIG32 || MFMA ? 1024 : 512);
    static constexpr int LDS = (F64 ? WIDE && !Y512 : BIG32) ? 131072 : 65536;
    static constexpr int TC_T = MAXT / TPT;
    static constexpr int CAP = C32 ? 32 : (256 / TPT) > 16 ? (256 / TPT) : 16;
    static constexpr int FULL = LDS / (N * int(sizeof(cx<T>)));
    static constexpr int A0 = TC_T < CAP ? TC_T : CAP;
    static constexpr int A1 = A0 < 2 * FULL ? A0 : 2 * FULL;
    static constexpr int TC = A1 < 1 ? 1 : A1;
    static constexpr int XP = TC > FULL ? 2 : 1;
};

// XP: LDS rounds per exchange.  1 = whole complex values, 2 = real then
// imaginary parts; the LDS tile is N*TC/XP complex values (padded).
// NT: non-temporal loads and stores of the lines (no reuse), for tilings in
// which every 128-byte line belongs to one tile (the host checks this).
// MF: 0 vector stages; 2 or 3 the first radix-16 stage on the matrix cores;
// -1 no transform (each element replaced by its conjugate): the same loads
// and stores as the pass, a yardstick for its memory-access ceiling.
template <typename T, int N, int TC, int XP, int S, int E = 16, int MF = 0, bool NT = false>
__global__ __launch_bounds__(TC * N / E) void k_strided(
    cx<T>* __restrict__ data, const cx<T>* __restrict__ tw, int64_t m_cols,
    int64_t tiles_m, line_map lm) {
    constexpr int TPT = N / E;
    constexpr bool SPLIT = XP == 2;
    static_assert(XP == 1 || XP == 2, "XP: whole values (1) or real/imaginary halves (2)");
    constexpr int RM = radix_cap<T, MF>();
    constexpr int PS = first_radix_shift<E, RM>::value;
    constexpr int NP = padded_len<N, PS>::value;
    __shared__ cx<T> lds[(NP * TC + XP - 1) / XP];
    using IX = idx_cols<TC, PS>;

    const int c = threadIdx.x % TC;
    const int t = threadIdx.x / TC;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t b = tile / tiles_m;
    const int64_t m0 = (tile - b * tiles_m) * TC;
    const int64_t m = m0 + c;
    const bool valid = m < m_cols;
    const int64_t ymask = (int64_t(1) << lm.lg_y) - 1;
    cx<T>* plane = data + (b >> lm.lg_bx) * lm.b_hi + (b & ((int64_t(1) << lm.lg_bx) - 1)) * lm.b_lo;
    auto off = [&](int64_t n) { return (n >> lm.lg_y) * lm.s_hi + (n & ymask) * lm.s_lo; };
    // Element n = t + i*TPT of a line: t < TPT and i*TPT have disjoint bits
    // (TPT a power of two), and off() adds over disjoint bit fields, so
    // off(n) = off(t) + off(i*TPT): a per-lane pointer plus an offset that
    // is the same for the whole workgroup, written in closed form as
    // off(i*TPT) = (i >> d) H + (i mod 2^d) Lo.  Lanes of the ragged last
    // tile read the last column instead (in bounds); their results are
    // dropped.
    constexpr int LGT = ilog2_c(TPT), LGE = ilog2_c(E);
    int d = 0;
    int64_t H = (int64_t(TPT) >> (lm.lg_y < LGT ? lm.lg_y : LGT)) * lm.s_hi, Lo = 0;
    if (lm.lg_y >= LGT) {
        d = lm.lg_y - LGT < LGE ? lm.lg_y - LGT : LGE;
        H = lm.s_hi;
        Lo = int64_t(TPT) * lm.s_lo;
    }
    auto uoff = [](int i, int d, int64_t H, int64_t Lo) {
        return int64_t(i >> d) * H + int64_t(i & ((1 << d) - 1)) * Lo;
    };
    int64_t lane_off = (valid ? m : m_cols - 1) + off(t);
    const cx<T>* lane = plane + lane_off;

    cx<T> a[E];
    if constexpr (MF < 0) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const cx<T>* p = lane + uoff(i, d, H, Lo);
            if constexpr (NT) {
                a[i].x = __builtin_nontemporal_load(&p->x);
                a[i].y = -__builtin_nontemporal_load(&p->y);
            } else {
                a[i] = conjg(*p);
            }
        }
        // all loads of the tile before any store, as in the transform
        __syncthreads();
    } else if constexpr (MF == 0) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const cx<T>* p = lane + uoff(i, d, H, Lo);
            if constexpr (NT) {
                a[i].x = __builtin_nontemporal_load(&p->x);
                a[i].y = __builtin_nontemporal_load(&p->y);
            } else {
                a[i] = *p;
            }
        }
        if constexpr (SPLIT)
            fft_regs<T, N, E, S, RM>(a, t, tw, 1,
                                     xch_split<T, IX>{reinterpret_cast<T*>(lds), IX{c}});
        else
            fft_regs<T, N, E, S, RM>(a, t, tw, 1, xch_full<T, IX>{lds, IX{c}});
    } else {
        // First radix-16 stage on the matrix cores.  The wave's 64 butterflies
        // (those of its own threads, j = t for thread (c, t)) go in two groups
        // of 32; lane (h, n) loads inputs 8h..8h+7 of butterfly 32g + n.
        static_assert(sizeof(T) == 4 && E == 16 && N >= 32, "MFMA stage: FP32, radix-16 first stage");
        const int lane = threadIdx.x & 63, h = lane >> 5;
        const int wbase = threadIdx.x & ~63;
        dft16_mfma<S, MF> dft;
        dft.init(lane);
        cx<float> y[2][8];
        int bc[2], bt[2];
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const int tid_b = wbase + 32 * g + (lane & 31);
            bc[g] = tid_b % TC;
            bt[g] = tid_b / TC;
            const bool vb = m0 + bc[g] < m_cols;
            cx<float> in[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int64_t n = bt[g] + (8 * h + j) * TPT;
                in[j] = vb ? plane[m0 + bc[g] + off(n)] : cx<float>{0.f, 0.f};
            }
            dft.run(in, y[g]);
        }
        // exchange: output r of butterfly (c_b, t_b) goes to position 16 t_b + r
        const IX pos_c{c};
        if constexpr (SPLIT) {
            T* buf = reinterpret_cast<T*>(lds);
#pragma unroll
            for (int part = 0; part < 2; ++part) {
#pragma unroll
                for (int g = 0; g < 2; ++g)
#pragma unroll
                    for (int v = 0; v < 8; ++v)
                        buf[IX{bc[g]}.at(xgeom<N, E, 1, 16>::template out_pad<PS>(bt[g], dft16_out_index(h, v) * (E / 16)))] =
                            part ? y[g][v].y : y[g][v].x;
                __syncthreads();
#pragma unroll
                for (int i = 0; i < E; ++i) {
                    const T val = buf[pos_c.at(xgeom<N, E, 1, 16>::template in_pad<PS>(t, i))];
                    if (part) a[i].y = val; else a[i].x = val;
                }
                __syncthreads();
            }
        } else {
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int v = 0; v < 8; ++v)
                    lds[IX{bc[g]}.at(xgeom<N, E, 1, 16>::template out_pad<PS>(bt[g], dft16_out_index(h, v) * (E / 16)))] = y[g][v];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < E; ++i) a[i] = lds[pos_c.at(xgeom<N, E, 1, 16>::template in_pad<PS>(t, i))];
            __syncthreads();
        }
        if constexpr (SPLIT)
            fft_from<T, N, E, S, 16>(a, t, tw, 1,
                                     xch_split<T, IX>{reinterpret_cast<T*>(lds), IX{c}});
        else
            fft_from<T, N, E, S, 16>(a, t, tw, 1, xch_full<T, IX>{lds, IX{c}});
    }
    if (!valid) return;
    // Opaque to the optimiser, so the store addresses are formed afresh
    // instead of keeping the E load addresses live through the transform.
    asm volatile("" : "+v"(lane_off));
    d = opaque_uniform(d);
    H = opaque_uniform(H);
    Lo = opaque_uniform(Lo);
    cx<T>* dst = plane + lane_off;
#pragma unroll
    for (int i = 0; i < E; ++i) {
        cx<T>* p = dst + uoff(i, d, H, Lo);
        if constexpr (NT) {
            __builtin_nontemporal_store(a[i].x, &p->x);
            __builtin_nontemporal_store(a[i].y, &p->y);
        } else {
            *p = a[i];
        }
    }
}

// ---------------------------------------------------------------- pack
template <typename T>
__global__ __launch_bounds__(kThreads) void k_pack(
    const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, int64_t len,
    int64_t blocks_per_chunk, int lg_x, int lg_p, int64_t n, int64_t y, int64_t k,
    bool to_send) {
    const int64_t chunk = blockIdx.x / blocks_per_chunk;
    const int64_t part = blockIdx.x - chunk * blocks_per_chunk;
    // chunk = (bb, j, xl) with xl fastest
    const int64_t xl = chunk & ((int64_t(1) << lg_x) - 1);
    const int64_t j = (chunk >> lg_x) & ((int64_t(1) << lg_p) - 1);
    const int64_t bb = chunk >> (lg_x + lg_p);
    const int64_t X = int64_t(1) << lg_x;
    const int64_t plane = bb * X * n * k;
    const int64_t nat = plane + (xl * n + j * y) * k;
    const int64_t snd = plane + (j * X + xl) * y * k;
    const cx<T>* s = src + (to_send ? nat : snd);
    cx<T>* d = dst + (to_send ? snd : nat);
    const int64_t step = blocks_per_chunk * kThreads;
    for (int64_t e = part * kThreads + threadIdx.x; e < len; e += step) d[e] = s[e];
}

// Row permutation copy: workgroup copies kRows rows, k values each.
constexpr int kPackRows = 4;
template <typename T>
__global__ __launch_bounds__(kThreads) void k_pack_rows(
    const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, int64_t rows, int64_t k,
    row_map map, bool to_send) {
#pragma unroll
    for (int i = 0; i < kPackRows; ++i) {
        const int64_t r = int64_t(blockIdx.x) * kPackRows + i;
        if (r >= rows) return;
        const int64_t q = map_row(r, map);
        const cx<T>* s = src + (to_send ? r : q) * k;
        cx<T>* d = dst + (to_send ? q : r) * k;
        for (int64_t e = threadIdx.x; e < k; e += kThreads) d[e] = s[e];
    }
}

// ---------------------------------------------------------------- copy
// Plain streaming copy, one 16-byte element per work-item and no reuse: the
// reference rate for what any pass can reach on contiguous memory.
__global__ __launch_bounds__(kThreads) void k_copy16(const uint4* __restrict__ src,
                                                     uint4* __restrict__ dst, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ---------------------------------------------------------------- launchers
// Grids are one-dimensional, and a dispatch carries its size in work-items
// as a 32-bit count: refuse grids beyond either limit.
static bool grid_fits(int64_t blocks, int64_t threads) {
    return blocks <= 0x7fffffff && blocks * threads <= int64_t(0xffffffff);
}

template <typename T, int N>
static hipError_t z_r2c_n(const void* in, void* out, const void* tw, int64_t rows,
                          row_map map, double me, double mi, hipStream_t s) {
    using C = zcfg<T, true, N>;
    using Z = zshape<N / 2, C::EMAX, C::THREADS>;
    const int64_t blocks = (rows + Z::RPB - 1) / Z::RPB;
    if (blocks == 0) return hipSuccess;
    if (!grid_fits(blocks, Z::NT)) return hipErrorInvalidValue;
    if (map.pencil)
        hipLaunchKernelGGL((k_z_r2c_pencil<T, N, C::EMAX, C::THREADS, C::REMAP>), dim3(blocks),
                           dim3(Z::NT), 0, s, static_cast<const T*>(in), static_cast<cx<T>*>(out),
                           static_cast<const cx<T>*>(tw), rows, map, T(me), T(mi));
    else if (in == out)
        hipLaunchKernelGGL((k_z_r2c_inplace<T, N, C::EMAX, C::THREADS, C::REMAP, C::NTS>),
                           dim3(blocks), dim3(Z::NT), 0, s, static_cast<const T*>(in),
                           static_cast<cx<T>*>(out), static_cast<const cx<T>*>(tw), rows, map,
                           T(me), T(mi));
    else
        hipLaunchKernelGGL((k_z_r2c<T, N, C::EMAX, C::THREADS, C::REMAP, C::NTS>), dim3(blocks),
                           dim3(Z::NT), 0, s, static_cast<const T*>(in), static_cast<cx<T>*>(out),
                           static_cast<const cx<T>*>(tw), rows, map, T(me), T(mi));
    return hipGetLastError();
}

template <typename T, int N>
static hipError_t z_c2r_n(const void* in, void* out, const void* tw, int64_t rows,
                          row_map map, double me, double mi, hipStream_t s) {
    using C = zcfg<T, false, N>;
    using Z = zshape<N / 2, C::EMAX, C::THREADS>;
    const int64_t blocks = (rows + Z::RPB - 1) / Z::RPB;
    if (blocks == 0) return hipSuccess;
    if (!grid_fits(blocks, Z::NT)) return hipErrorInvalidValue;
    if (map.pencil)
        hipLaunchKernelGGL((k_z_c2r_pencil<T, N, C::EMAX, C::THREADS, C::REMAP, C::NTS>),
                           dim3(blocks), dim3(Z::NT), 0, s, static_cast<const cx<T>*>(in),
                           static_cast<T*>(out), static_cast<const cx<T>*>(tw), rows, map,
                           T(me), T(mi));
    else if (in == out)
        hipLaunchKernelGGL((k_z_c2r_inplace<T, N, C::EMAX, C::THREADS, C::REMAP, C::NTS>),
                           dim3(blocks), dim3(Z::NT), 0, s, static_cast<const cx<T>*>(in),
                           static_cast<T*>(out), static_cast<const cx<T>*>(tw), rows, map,
                           T(me), T(mi));
    else
        hipLaunchKernelGGL((k_z_c2r<T, N, C::EMAX, C::THREADS, C::REMAP, C::NTS>), dim3(blocks),
                           dim3(Z::NT), 0, s, static_cast<const cx<T>*>(in), static_cast<T*>(out),
                           static_cast<const cx<T>*>(tw), rows, map, T(me), T(mi));
    return hipGetLastError();
}

// True when each tile of a multiple of `la` columns covers whole lines of
// `la` elements: the base is 128-byte aligned and every offset of the
// layout, and the column count, are multiples of `la`.
static bool whole_lines(const void* data, int64_t m_cols, const line_map& lm, int64_t la) {
    return reinterpret_cast<uintptr_t>(data) % 128 == 0 && m_cols % la == 0 &&
           lm.b_hi % la == 0 && lm.b_lo % la == 0 && lm.s_hi % la == 0 && lm.s_lo % la == 0;
}

template <typename T, int N, int AX, int MF>
static hipError_t strided_ax(int sign, void* data, const void* tw, int64_t m_cols,
                             int64_t n_b, line_map lm, hipStream_t s) {
    using SH = sshape<T, N, AX, (MF > 0)>;
    constexpr int TC = SH::TC;
    const int64_t tiles_m = (m_cols + TC - 1) / TC;
    const int64_t blocks = tiles_m * n_b;
    if (blocks == 0) return hipSuccess;
    if (!grid_fits(blocks, TC * SH::TPT)) return hipErrorInvalidValue;
    const dim3 threads(TC * SH::TPT);
    // x lines stream through non-temporally when every tile owns whole
    // 128-byte lines: at 1024^3 2% faster in FP64 and 4% in FP32, at 2048^3
    // 8% faster in FP32 but 5% slower in FP64 (one 512-thread workgroup per
    // CU), so FP64 uses it for N = 512 and 1024 only, FP32 from N = 256.
    // Where neighbouring tiles share lines, as in the y passes, the hint
    // makes them travel twice (15-50% slower).
    if constexpr (AX == 1 && MF <= 0 && (N >= 512 || (sizeof(T) == 4 && N == 256)) &&
                  (sizeof(T) == 4 || N <= 1024) && (TC * sizeof(cx<T>)) % 128 == 0) {
        if (whole_lines(data, m_cols, lm, 128 / int64_t(sizeof(cx<T>)))) {
            if (MF < 0 || sign < 0)
                hipLaunchKernelGGL((k_strided<T, N, TC, SH::XP, -1, SH::E, MF, true>), dim3(blocks),
                                   threads, 0, s, static_cast<cx<T>*>(data),
                                   static_cast<const cx<T>*>(tw), m_cols, tiles_m, lm);
            else if constexpr (MF == 0)
                hipLaunchKernelGGL((k_strided<T, N, TC, SH::XP, +1, SH::E, 0, true>), dim3(blocks),
                                   threads, 0, s, static_cast<cx<T>*>(data),
                                   static_cast<const cx<T>*>(tw), m_cols, tiles_m, lm);
            return hipGetLastError();
        }
    }
    if (MF < 0 || sign < 0)
        hipLaunchKernelGGL((k_strided<T, N, TC, SH::XP, -1, SH::E, MF>), dim3(blocks), threads,
                           0, s, static_cast<cx<T>*>(data), static_cast<const cx<T>*>(tw),
                           m_cols, tiles_m, lm);
    else if constexpr (MF >= 0)
        hipLaunchKernelGGL((k_strided<T, N, TC, SH::XP, +1, SH::E, MF>), dim3(blocks), threads,
                           0, s, static_cast<cx<T>*>(data), static_cast<const cx<T>*>(tw),
                           m_cols, tiles_m, lm);
    return hipGetLastError();
}

template <typename T, int N>
static hipError_t strided_n(int axis, int mfma_terms, int sign, void* data, const void* tw,
                            int64_t m_cols, int64_t n_b, line_map lm, hipStream_t s) {
    if (mfma_terms == -1)
        return axis == 0 ? strided_ax<T, N, 0, -1>(sign, data, tw, m_cols, n_b, lm, s)
                         : strided_ax<T, N, 1, -1>(sign, data, tw, m_cols, n_b, lm, s);
    if constexpr (sizeof(T) == 4 && N >= 32) {
        if (mfma_terms == 2)
            return axis == 0 ? strided_ax<T, N, 0, 2>(sign, data, tw, m_cols, n_b, lm, s)
                             : strided_ax<T, N, 1, 2>(sign, data, tw, m_cols, n_b, lm, s);
        if (mfma_terms == 3)
            return axis == 0 ? strided_ax<T, N, 0, 3>(sign, data, tw, m_cols, n_b, lm, s)
                             : strided_ax<T, N, 1, 3>(sign, data, tw, m_cols, n_b, lm, s);
    }
    if (mfma_terms != 0) return hipErrorInvalidValue;
    if (axis == 0) return strided_ax<T, N, 0, 0>(sign, data, tw, m_cols, n_b, lm, s);
    return strided_ax<T, N, 1, 0>(sign, data, tw, m_cols, n_b, lm, s);
}

#define GFFT_DISPATCH_N(FN, T, ...)                 \
    switch (n) {                                    \
        case 16: return FN<T, 16>(__VA_ARGS__);     \
        case 32: return FN<T, 32>(__VA_ARGS__);     \
        case 64: return FN<T, 64>(__VA_ARGS__);     \
        case 128: return FN<T, 128>(__VA_ARGS__);   \
        case 256: return FN<T, 256>(__VA_ARGS__);   \
        case 512: return FN<T, 512>(__VA_ARGS__);   \
        case 1024: return FN<T, 1024>(__VA_ARGS__); \
        case 2048: return FN<T, 2048>(__VA_ARGS__); \
        case 4096: return FN<T, 4096>(__VA_ARGS__); \
        default: return hipErrorInvalidValue;       \
    }

hipError_t launch_z_r2c(bool f64, int n, const void* in, void* out, const void* tw,
                        int64_t rows, row_map map, double me, double mi, hipStream_t s) {
    if (f64) { GFFT_DISPATCH_N(z_r2c_n, double, in, out, tw, rows, map, me, mi, s) }
    GFFT_DISPATCH_N(z_r2c_n, float, in, out, tw, rows, map, me, mi, s)
}

hipError_t launch_z_c2r(bool f64, int n, const void* in, void* out, const void* tw,
                        int64_t rows, row_map map, double me, double mi, hipStream_t s) {
    if (f64) { GFFT_DISPATCH_N(z_c2r_n, double, in, out, tw, rows, map, me, mi, s) }
    GFFT_DISPATCH_N(z_c2r_n, float, in, out, tw, rows, map, me, mi, s)
}

hipError_t launch_strided(bool f64, int n, int axis, int mfma_terms, int sign, void* data,
                          const void* tw, int64_t m_cols, int64_t n_b, line_map lm,
                          hipStream_t s) {
    if (f64) { GFFT_DISPATCH_N(strided_n, double, axis, mfma_terms, sign, data, tw, m_cols, n_b, lm, s) }
    GFFT_DISPATCH_N(strided_n, float, axis, mfma_terms, sign, data, tw, m_cols, n_b, lm, s)
}

hipError_t launch_pack(bool f64, const void* src, void* dst, int64_t chunks, int lg_x,
                       int lg_p, int64_t n, int64_t y, int64_t k, bool to_send,
                       hipStream_t s) {
    const int64_t len = y * k;
    int64_t bpc = (len + kThreads * 4 - 1) / (kThreads * 4);
    // k_pack strides over its chunk, so fewer blocks per chunk keep very
    // large grids within the dispatch's 32-bit work-item count
    const int64_t cap = chunks > 0 ? int64_t(0xffffffff) / (chunks * kThreads) : 1;
    if (bpc > cap) bpc = cap;
    if (bpc < 1) bpc = 1;
    const int64_t blocks = chunks * bpc;
    if (blocks == 0 || len == 0) return hipSuccess;
    if (!grid_fits(blocks, kThreads)) return hipErrorInvalidValue;
    if (f64)
        hipLaunchKernelGGL((k_pack<double>), dim3(blocks), dim3(kThreads), 0, s,
                           static_cast<const cx<double>*>(src), static_cast<cx<double>*>(dst),
                           len, bpc, lg_x, lg_p, n, y, k, to_send);
    else
        hipLaunchKernelGGL((k_pack<float>), dim3(blocks), dim3(kThreads), 0, s,
                           static_cast<const cx<float>*>(src), static_cast<cx<float>*>(dst),
                           len, bpc, lg_x, lg_p, n, y, k, to_send);
    return hipGetLastError();
}

hipError_t launch_pack_rows(bool f64, const void* src, void* dst, int64_t rows, int64_t k,
                            row_map map, bool to_send, hipStream_t s) {
    const int64_t blocks = (rows + kPackRows - 1) / kPackRows;
    if (blocks == 0 || k == 0) return hipSuccess;
    if (!grid_fits(blocks, kThreads)) return hipErrorInvalidValue;
    if (f64)
        hipLaunchKernelGGL((k_pack_rows<double>), dim3(blocks), dim3(kThreads), 0, s,
                           static_cast<const cx<double>*>(src), static_cast<cx<double>*>(dst),
                           rows, k, map, to_send);
    else
        hipLaunchKernelGGL((k_pack_rows<float>), dim3(blocks), dim3(kThreads), 0, s,
                           static_cast<const cx<float>*>(src), static_cast<cx<float>*>(dst),
                           rows, k, map, to_send);
    return hipGetLastError();
}

template <int N>
static hipError_t plane_n(bool forward, const void* in, void* out, const void* tw, int64_t planes,
                          row_map map, double me, double mi, hipStream_t s) {
    if (planes == 0) return hipSuccess;
    if (!grid_fits(planes, plane_shape<N>::NT)) return hipErrorInvalidValue;
    if (forward) {
        hipLaunchKernelGGL(k_plane_r2c<N>, dim3(planes), dim3(plane_shape<N>::NT), 0, s,
                           static_cast<const float*>(in), static_cast<cx<float>*>(out),
                           static_cast<const cx<float>*>(tw), planes, map, float(me), float(mi));
    } else {
        if constexpr (N <= 128) {
            hipLaunchKernelGGL(k_plane_c2r<N>, dim3(planes), dim3(plane_shape<N>::NT), 0, s,
                               static_cast<const cx<float>*>(in), static_cast<float*>(out),
                               static_cast<const cx<float>*>(tw), planes, map, float(me),
                               float(mi));
        } else {
            return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

// Measured against the separate passes over 537 MB of FP32 reals (a pair is
// forward + inverse): N = 64 1.10 vs 2.14 ms per pair, N = 128 1.22 vs
// 1.57 ms; at N = 256 the plane fills half the register file, one workgroup
// runs per CU, and only the forward gains (0.65 vs 0.73 ms with the x pass;
// the inverse takes 0.81 vs 0.72 ms), so the inverse keeps the separate
// passes there.
bool plane_supported(bool f64, int n, bool forward) {
    return !f64 && (n == 64 || n == 128 || (forward && n == 256));
}

hipError_t launch_plane(bool f64, bool forward, int n, const void* in, void* out, const void* tw,
                        int64_t planes, row_map map, double me, double mi, hipStream_t s) {
    if (!plane_supported(f64, n, forward)) return hipErrorInvalidValue;
    switch (n) {
        case 64: return plane_n<64>(forward, in, out, tw, planes, map, me, mi, s);
        case 128: return plane_n<128>(forward, in, out, tw, planes, map, me, mi, s);
        case 256: return plane_n<256>(forward, in, out, tw, planes, map, me, mi, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_copy16(const void* src, void* dst, int64_t n16, hipStream_t s) {
    // at most 2^31 work-items per dispatch; longer copies take several
    constexpr int64_t kMax = int64_t(1) << 31;
    for (int64_t done = 0; done < n16; done += kMax) {
        const int64_t len = n16 - done < kMax ? n16 - done : kMax;
        const int64_t blocks = (len + kThreads - 1) / kThreads;
        hipLaunchKernelGGL(k_copy16, dim3(blocks), dim3(kThreads), 0, s,
                           static_cast<const uint4*>(src) + done, static_cast<uint4*>(dst) + done,
                           len);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace gfft
