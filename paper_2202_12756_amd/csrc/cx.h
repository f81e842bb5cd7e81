// Complex arithmetic and in-register DFT butterflies for gfx950.
//
// A DFT of radix R with sign S computes y[k] = sum_n a[n] w^(n k) with
// w = exp(S 2 pi i / R): S = -1 is the forward transform of the forward
// equation (section 2), S = +1 the inverse.  Radix 8 and 16 are split into
// radix-4/2 pieces by the Cooley-Tukey index map (decimation in time).
#pragma once

#include <hip/hip_runtime.h>

namespace gfft {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> scal(cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) { return {a.x, -a.y}; }

// a * (S i)
template <int S, typename T>
__device__ __forceinline__ cx<T> mul_si(cx<T> a) {
    return S < 0 ? cx<T>{a.y, -a.x} : cx<T>{-a.y, a.x};
}

// Multiply by a table twiddle exp(-2 pi i m / N) (S = -1) or its conjugate.
template <int S, typename T>
__device__ __forceinline__ cx<T> twiddle(cx<T> a, cx<T> w) {
    return S < 0 ? cmul(a, w) : cmulc(a, w);
}

template <typename T> struct k_ {
    static constexpr T r2 = T(0.70710678118654752440084436210484903928);  // cos(pi/4)
    static constexpr T c8 = T(0.92387953251128675612818318939678828682);  // cos(pi/8)
    static constexpr T s8 = T(0.38268343236508977172845998403039886676);  // sin(pi/8)
};

// a * exp(S i pi/4) = a (1 + S i)/sqrt2
template <int S, typename T>
__device__ __forceinline__ cx<T> mul_w8_1(cx<T> a) {
    return {(a.x - S * a.y) * k_<T>::r2, (a.y + S * a.x) * k_<T>::r2};
}
// a * exp(S i 3pi/4) = a (-1 + S i)/sqrt2
template <int S, typename T>
__device__ __forceinline__ cx<T> mul_w8_3(cx<T> a) {
    return {(-a.x - S * a.y) * k_<T>::r2, (S * a.x - a.y) * k_<T>::r2};
}
// a * (c + S i s)
template <int S, typename T>
__device__ __forceinline__ cx<T> mul_cs(cx<T> a, T c, T s) {
    return {a.x * c - S * a.y * s, a.y * c + S * a.x * s};
}

template <int S, typename T>
__device__ __forceinline__ void dft2(cx<T>& a0, cx<T>& a1) {
    cx<T> t = a0 - a1;
    a0 = a0 + a1;
    a1 = t;
}

template <int S, typename T>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
    cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = mul_si<S>(a1 - a3);
    a0 = t0 + t2;
    a2 = t0 - t2;
    a1 = t1 + t3;
    a3 = t1 - t3;
}

// Radix 8: y_k = E_k + w8^k O_k, y_{k+4} = E_k - w8^k O_k with E, O the
// 4-point DFTs of the even and odd inputs.
template <int S, typename T>
__device__ __forceinline__ void dft8(cx<T>* a) {
    dft4<S>(a[0], a[2], a[4], a[6]);
    dft4<S>(a[1], a[3], a[5], a[7]);
    cx<T> o1 = mul_w8_1<S>(a[3]);   // O_1 sits in a[3] after the in-place dft4
    cx<T> o2 = mul_si<S>(a[5]);     // O_2 in a[5]
    cx<T> o3 = mul_w8_3<S>(a[7]);   // O_3 in a[7]
    cx<T> o0 = a[1];
    cx<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
    a[0] = e0 + o0; a[4] = e0 - o0;
    a[1] = e1 + o1; a[5] = e1 - o1;
    a[2] = e2 + o2; a[6] = e2 - o2;
    a[3] = e3 + o3; a[7] = e3 - o3;
}

// Radix 16 as 4 x 4: with n = 4 n1 + n2 and k = k1 + 4 k2,
// y_k = sum_n2 w4^(n2 k2) [w16^(n2 k1) sum_n1 a_(4 n1 + n2) w4^(n1 k1)].
template <int S, typename T>
__device__ __forceinline__ void dft16(cx<T>* a) {
    // inner 4-point DFTs over n1 for each n2: inputs a[n2], a[4+n2], a[8+n2], a[12+n2]
    // afterwards a[n2 + 4 k1] holds B[n2][k1]
    dft4<S>(a[0], a[4], a[8], a[12]);
    dft4<S>(a[1], a[5], a[9], a[13]);
    dft4<S>(a[2], a[6], a[10], a[14]);
    dft4<S>(a[3], a[7], a[11], a[15]);
    // twiddles w16^(n2 k1) on B[n2][k1] = a[n2 + 4 k1]
    const T c = k_<T>::c8, s = k_<T>::s8;
    a[5] = mul_cs<S>(a[5], c, s);          // n2=1,k1=1: m=1
    a[9] = mul_w8_1<S>(a[9]);              // n2=1,k1=2: m=2
    a[13] = mul_cs<S>(a[13], s, c);        // n2=1,k1=3: m=3
    a[6] = mul_w8_1<S>(a[6]);              // n2=2,k1=1: m=2
    a[10] = mul_si<S>(a[10]);              // n2=2,k1=2: m=4
    a[14] = mul_w8_3<S>(a[14]);            // n2=2,k1=3: m=6
    a[7] = mul_cs<S>(a[7], s, c);          // n2=3,k1=1: m=3
    a[11] = mul_w8_3<S>(a[11]);            // n2=3,k1=2: m=6
    a[15] = mul_cs<S>(a[15], -c, -s);      // n2=3,k1=3: m=9
    // outer 4-point DFTs over n2 for each k1: output k = k1 + 4 k2
    dft4<S>(a[0], a[1], a[2], a[3]);
    dft4<S>(a[4], a[5], a[6], a[7]);
    dft4<S>(a[8], a[9], a[10], a[11]);
    dft4<S>(a[12], a[13], a[14], a[15]);
    // now a[4 k1 + k2] = y[k1 + 4 k2]: transpose the 4x4 index
    cx<T> t;
    t = a[1]; a[1] = a[4]; a[4] = t;
    t = a[2]; a[2] = a[8]; a[8] = t;
    t = a[3]; a[3] = a[12]; a[12] = t;
    t = a[6]; a[6] = a[9]; a[9] = t;
    t = a[7]; a[7] = a[13]; a[13] = t;
    t = a[11]; a[11] = a[14]; a[14] = t;
}

// cos and sin of pi/16 and 3 pi/16 (nested half-angle formulas:
// cos(pi/16) = sqrt(2 + sqrt(2 + sqrt 2)) / 2, and so on)
template <typename T> struct k32_ {
    static constexpr T c1 = T(0.98078528040323044912618223613423903697);
    static constexpr T s1 = T(0.19509032201612826784828486847702224092);
    static constexpr T c3 = T(0.83146961230254523707878837761790575673);
    static constexpr T s3 = T(0.55557023301960222474283081394853287437);
};

// Radix 32 as 2 x 16 (decimation in time): with E and O the 16-point DFTs of
// the even and odd inputs, y_k = E_k + w32^k O_k and y_(k+16) = E_k - w32^k O_k,
// w32^k = cos(pi k/16) + S i sin(pi k/16).
template <int S, typename T>
__device__ __forceinline__ void dft32(cx<T>* a) {
    cx<T> e[16], o[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        e[i] = a[2 * i];
        o[i] = a[2 * i + 1];
    }
    dft16<S>(e);
    dft16<S>(o);
    const T c1 = k32_<T>::c1, s1 = k32_<T>::s1, c3 = k32_<T>::c3, s3 = k32_<T>::s3;
    const T c2 = k_<T>::c8, s2 = k_<T>::s8;
    o[1] = mul_cs<S>(o[1], c1, s1);
    o[2] = mul_cs<S>(o[2], c2, s2);
    o[3] = mul_cs<S>(o[3], c3, s3);
    o[4] = mul_w8_1<S>(o[4]);
    o[5] = mul_cs<S>(o[5], s3, c3);
    o[6] = mul_cs<S>(o[6], s2, c2);
    o[7] = mul_cs<S>(o[7], s1, c1);
    o[8] = mul_si<S>(o[8]);
    o[9] = mul_cs<S>(o[9], -s1, c1);
    o[10] = mul_cs<S>(o[10], -s2, c2);
    o[11] = mul_cs<S>(o[11], -s3, c3);
    o[12] = mul_w8_3<S>(o[12]);
    o[13] = mul_cs<S>(o[13], -c3, s3);
    o[14] = mul_cs<S>(o[14], -c2, s2);
    o[15] = mul_cs<S>(o[15], -c1, s1);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        a[k] = e[k] + o[k];
        a[k + 16] = e[k] - o[k];
    }
}

template <int R, int S, typename T>
__device__ __forceinline__ void dft(cx<T>* a) {
    if constexpr (R == 2) {
        dft2<S>(a[0], a[1]);
    } else if constexpr (R == 4) {
        dft4<S>(a[0], a[1], a[2], a[3]);
    } else if constexpr (R == 8) {
        dft8<S>(a);
    } else if constexpr (R == 16) {
        dft16<S>(a);
    } else if constexpr (R == 32) {
        dft32<S>(a);
    } else {
        static_assert(R == 1, "radix must be 1, 2, 4, 8, 16 or 32");
    }
}

}  // namespace gfft
