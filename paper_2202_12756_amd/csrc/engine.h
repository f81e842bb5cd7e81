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

// Radix of the stage that starts at span L: E while the remaining length
// allows, then whatever is left (N, E powers of two).
template <int N, int E, int L>
struct stage_radix {
    static constexpr int value = (N / L) >= E ? E : (N / L);
};

// LDS views.  `put`/`get` address element `pos` of the transform this
// thread works on.
//   column tile: element (pos, c) at buf[pos*TC + c]      (strided axes)
//   row tile:    element (row, pos) at buf[row*RS + pos]   (contiguous rows)
template <typename T, int TC>
struct lds_cols {
    cx<T>* buf;
    int c;
    __device__ __forceinline__ void put(int pos, cx<T> v) const { buf[pos * TC + c] = v; }
    __device__ __forceinline__ cx<T> get(int pos) const { return buf[pos * TC + c]; }
};

template <typename T>
struct lds_rows {
    cx<T>* buf;  // already offset to this thread's row
    __device__ __forceinline__ void put(int pos, cx<T> v) const { buf[pos] = v; }
    __device__ __forceinline__ cx<T> get(int pos) const { return buf[pos]; }
};

// Run the stages from span L to the end.  `tw` is a table of
// W_Ntab^m (m = 0..Ntab-1) with Ntab = N * tws; entry idx*tws is W_N^idx.
template <typename T, int N, int E, int S, int L, class Lds>
__device__ __forceinline__ void fft_from(cx<T> (&a)[E], int t,
                                         const cx<T>* __restrict__ tw, int tws,
                                         const Lds& lds) {
    constexpr int R = stage_radix<N, E, L>::value;
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
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) a[q + r * NB] = b[r];
        } else {
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds.put(base + r * L, b[r]);
        }
    }
    if constexpr (!LAST) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m) a[m] = lds.get(t + m * TPT);
        __syncthreads();
        fft_from<T, N, E, S, L * R>(a, t, tw, tws, lds);
    }
}

template <typename T, int N, int E, int S, class Lds>
__device__ __forceinline__ void fft_regs(cx<T> (&a)[E], int t,
                                         const cx<T>* __restrict__ tw, int tws,
                                         const Lds& lds) {
    fft_from<T, N, E, S, 1>(a, t, tw, tws, lds);
}

}  // namespace gfft
