// Register-resident Stockham FFT with LDS exchanges between radix stages.
//
// One transform of length N is spread over TPT = N/E threads that each hold
// E elements in registers.  Thread t always holds the elements at positions
// t + m*TPT (m = 0..E-1) of the current stage's input, so that the first
// stage can load straight from global memory and the last stage can store
// straight to it: across consecutive threads the positions are consecutive.
//
// Stage with span L (product of the radices already applied) and radix R
// (the self-sorting Stockham formulation of the Cooley-Tukey FFT): for each
// butterfly j in [0, N/R) with k = j mod L,
//   inputs   x[j + r N/R]                        r = 0..R-1
//   twiddle  x[j + r N/R] *= W_N^(r k N/(L R))   (W_N = exp(-2 pi i/N))
//   DFT_R over r
//   outputs  y[(j - k) R + k + r L]
// After the last stage (L R = N) the outputs are in natural order, and they
// fall on the same positions the thread read, so no exchange follows it.
#pragma once

#include "cx.h"

namespace gfft {

// Radix of the stage that starts at span L: min(E, RM) while the remaining
// length allows, then whatever is left (N, E, RM powers of two; RM = 16 or
// 32).  With E > RM a thread runs E/RM butterflies per stage.
template <int N, int E, int L, int RM = 16>
struct stage_radix {
    static constexpr int RMAX = E < RM ? E : RM;
    static constexpr int value = (N / L) >= RMAX ? RMAX : (N / L);
};

// Where element `pos` of this thread's transform lives in an LDS buffer.
// The first exchange sends consecutive threads' outputs R0 positions apart
// (R0 = 2^PS, the first radix), which would put them in the same LDS banks;
// one padding position after every R0 positions staggers them:
// pad(pos) = pos + (pos >> PS).
//   columns: TC transforms side by side, element (pos, c) at pad(pos)*TC + c
//   rows:    one transform per row, element pos at off + pad(pos)
template <int PS>
__device__ __forceinline__ int lds_pad(int pos) {
    if constexpr (PS > 0) return pos + (pos >> PS);
    else return pos;
}
// Positions a transform of length N occupies once padded.
template <int N, int PS>
struct padded_len {
    static constexpr int value = PS > 0 ? N + (N >> PS) : N;
};
template <int TC, int PS = 0>
struct idx_cols {
    static constexpr int SHIFT = PS;
    int c;
    __device__ __forceinline__ int at(int padded) const { return padded * TC + c; }
    __device__ __forceinline__ int operator()(int pos) const { return at(lds_pad<PS>(pos)); }
};
template <int PS = 0>
struct idx_rows {
    static constexpr int SHIFT = PS;
    int off;
    __device__ __forceinline__ int at(int padded) const { return off + padded; }
    __device__ __forceinline__ int operator()(int pos) const { return at(lds_pad<PS>(pos)); }
};
// log2 of the first radix for E elements per thread (radix cap RM)
template <int E, int RM = 16>
struct first_radix_shift {
    static constexpr int R0 = E < RM ? E : RM;
    static constexpr int value =
        R0 >= 32 ? 5 : R0 >= 16 ? 4 : R0 >= 8 ? 3 : R0 >= 4 ? 2 : R0 >= 2 ? 1 : 0;
};

// Exchange after a stage: every output slot q + r*NB goes to position
// (j - k) R + k + r L; then slot m is reloaded from position t + m*TPT.
// Padded positions are formed so that they stay affine in r and m (a base
// per butterfly plus compile-time steps): with R0 = 2^PS, the first stage
// (L = 1, R = R0) writes j (R0 + 1) + r, later stages (L a multiple of R0)
// write pad((j-k)R + k) + r (L + L/R0), and reads are
// pad(t) + m (TPT + TPT/R0) when R0 divides TPT.
template <int N, int E, int L, int R>
struct xgeom {
    static constexpr int NB = E / R, TPT = N / E;
    __device__ __forceinline__ static int out_pos(int t, int s) {
        const int q = s % NB, r = s / NB;
        const int j = t + q * TPT, k = j & (L - 1);
        return (j - k) * R + k + r * L;
    }
    // padded position of output slot s
    template <int PS>
    __device__ __forceinline__ static int out_pad(int t, int s) {
        const int q = s % NB, r = s / NB;
        const int j = t + q * TPT;
        if constexpr (PS == 0) {
            const int k = j & (L - 1);
            return (j - k) * R + k + r * L;
        } else if constexpr (L == 1 && R == (1 << PS)) {
            return j * (R + 1) + r;
        } else if constexpr (L % (1 << PS) == 0) {
            const int k = j & (L - 1);
            return lds_pad<PS>((j - k) * R + k) + r * (L + (L >> PS));
        } else {
            return lds_pad<PS>(out_pos(t, s));
        }
    }
    // padded position of input slot m
    template <int PS>
    __device__ __forceinline__ static int in_pad(int t, int m) {
        if constexpr (PS == 0) return t + m * TPT;
        else if constexpr (TPT % (1 << PS) == 0) return lds_pad<PS>(t) + m * (TPT + (TPT >> PS));
        else return lds_pad<PS>(t + m * TPT);
    }
};

// Whole complex values through a buffer of N*width complex entries.
template <typename T, class Idx>
struct xch_full {
    cx<T>* buf;
    Idx idx;
    template <int N, int E, int L, int R>
    __device__ __forceinline__ void run(cx<T> (&a)[E], int t) const {
        using G = xgeom<N, E, L, R>;
        constexpr int PS = Idx::SHIFT;
#pragma unroll
        for (int s = 0; s < E; ++s) buf[idx.at(G::template out_pad<PS>(t, s))] = a[s];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m) a[m] = buf[idx.at(G::template in_pad<PS>(t, m))];
        __syncthreads();
    }
};

// Real parts, then imaginary parts, through a buffer of half the size.
template <typename T, class Idx>
struct xch_split {
    T* buf;
    Idx idx;
    template <int N, int E, int L, int R>
    __device__ __forceinline__ void run(cx<T> (&a)[E], int t) const {
        using G = xgeom<N, E, L, R>;
        constexpr int PS = Idx::SHIFT;
#pragma unroll
        for (int s = 0; s < E; ++s) buf[idx.at(G::template out_pad<PS>(t, s))] = a[s].x;
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m) a[m].x = buf[idx.at(G::template in_pad<PS>(t, m))];
        __syncthreads();
#pragma unroll
        for (int s = 0; s < E; ++s) buf[idx.at(G::template out_pad<PS>(t, s))] = a[s].y;
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m) a[m].y = buf[idx.at(G::template in_pad<PS>(t, m))];
        __syncthreads();
    }
};

// Run the stages from span L to the end.  `tw` is a table of
// W_Ntab^m (m = 0..Ntab-1) with Ntab = N * tws; entry idx*tws is W_N^idx.
template <typename T, int N, int E, int S, int L, int RM = 16, class X>
__device__ __forceinline__ void fft_from(cx<T> (&a)[E], int t,
                                         const cx<T>* __restrict__ tw, int tws,
                                         const X& xch) {
    constexpr int R = stage_radix<N, E, L, RM>::value;
    constexpr int NB = E / R;       // butterflies per thread
    constexpr int TPT = N / E;      // threads per transform
    constexpr bool LAST = (L * R == N);
    static_assert(E % R == 0 && N % (L * R) == 0, "bad stage shape");

#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int j = t + q * TPT;
        const int k = j & (L - 1);
        cx<T> b[R];
#pragma unroll
        for (int r = 0; r < R; ++r) b[r] = a[q + r * NB];
        if constexpr (L > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const int idx = r * k * (N / (L * R));
                b[r] = twiddle<S>(b[r], tw[idx * tws]);
            }
        }
        dft<R, S>(b);
#pragma unroll
        for (int r = 0; r < R; ++r) a[q + r * NB] = b[r];
    }
    if constexpr (!LAST) {
        xch.template run<N, E, L, R>(a, t);
        fft_from<T, N, E, S, L * R, RM>(a, t, tw, tws, xch);
    }
}

template <typename T, int N, int E, int S, int RM = 16, class X>
__device__ __forceinline__ void fft_regs(cx<T> (&a)[E], int t,
                                         const cx<T>* __restrict__ tw, int tws,
                                         const X& xch) {
    fft_from<T, N, E, S, 1, RM>(a, t, tw, tws, xch);
}

}  // namespace gfft
