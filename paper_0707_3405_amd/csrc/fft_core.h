// Register-level DFT butterflies and the two-stage in-LDS FFT used by the
// plane-wave H.X apply.
//
// A length-N transform (N = R1 * R2, both factors products of 2, 3, 5 and at
// most 16; the split is a type P = Split<N, R2>) is done in place in LDS in
// two stages separated by one barrier:
//
//   dit  (natural order in -> digit-reversed out):
//     stage A, item n2:  DFT_R1 over x[n1*R2 + n2], twiddle W_N^{S n2 k1},
//                        write back to position k1*R2 + n2
//     stage B, item k1:  DFT_R2 over positions k1*R2 + n2 -> X[k1 + R1 k2]
//                        stored at position k1*R2 + k2
//   dif  (digit-reversed in -> natural out) is the adjoint sequence:
//     stage B', item k1: DFT_R2 over positions k1*R2 + k2 -> index n2
//     stage A', item n2: twiddle W_N^{S n2 k1}, DFT_R1 over k1 -> n1,
//                        natural position n1*R2 + n2
//
// with W_N = exp(2 pi i / N) and S = +1 (grid -> real space, no scale) or -1.
// Because both stages read and write the same positions, no second buffer and
// no extra barrier are needed; consumers of a dit result index it through
// digit_rev().
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "pw_internal.h"

namespace pw {
namespace fft {

// ---- compile-time trigonometry (Taylor series on [0, pi/4]) ---------------
constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double x) {
    double term = x, sum = x;
    for (int k = 1; k < 20; ++k) {
        term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double taylor_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 20; ++k) {
        term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}
struct SinCos {
    double s, c;
};
// sin and cos of 2 pi num / den by quadrant and octant reduction.
constexpr SinCos sincos2pi(long num, long den) {
    long r = ((num % den) + den) % den;
    long q = (4 * r) / den;          // quadrant
    long rem = 4 * r - q * den;      // angle within quadrant = (pi/2) rem / den
    double sphi = 0, cphi = 1;
    if (2 * rem <= den) {
        double phi = (kPi / 2) * double(rem) / double(den);
        sphi = taylor_sin(phi);
        cphi = taylor_cos(phi);
    } else {
        double phi = (kPi / 2) * double(den - rem) / double(den);
        sphi = taylor_cos(phi);
        cphi = taylor_sin(phi);
    }
    switch (q) {
        case 0: return {sphi, cphi};
        case 1: return {cphi, -sphi};
        case 2: return {-sphi, -cphi};
        default: return {-cphi, sphi};
    }
}

template <int Begin, int End, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (Begin < End) {
        f(std::integral_constant<int, Begin>{});
        static_for<Begin + 1, End>(static_cast<F &&>(f));
    }
}

// ---- complex helpers --------------------------------------------------------
template <class T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <class T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <class T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class T>
__device__ __forceinline__ cpx<T> cscale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
// S * i * z
template <int S, class T>
__device__ __forceinline__ cpx<T> mul_si(cpx<T> z) {
    if constexpr (S > 0) return {-z.y, z.x};
    else return {z.y, -z.x};
}
// z * exp(S 2 pi i NUM / DEN), trivial angles special-cased.
template <int S, long NUM, long DEN, class T>
__device__ __forceinline__ cpx<T> twc(cpx<T> z) {
    constexpr long r = ((NUM % DEN) + DEN) % DEN;
    if constexpr (r == 0) {
        return z;
    } else if constexpr (4 * r == DEN) {
        return mul_si<S>(z);
    } else if constexpr (2 * r == DEN) {
        return {-z.x, -z.y};
    } else if constexpr (4 * r == 3 * DEN) {
        return mul_si<-S>(z);
    } else {
        constexpr SinCos w = sincos2pi(r, DEN);
        constexpr T c = T(w.c);
        constexpr T s = T(S * w.s);
        return {z.x * c - z.y * s, z.x * s + z.y * c};
    }
}

// ---- small DFTs in registers: X[k] = sum_n x[n] exp(S 2 pi i n k / R) ------
constexpr int first_factor(int r) {
    return (r % 4 == 0 && r > 4) ? 4 : (r % 2 == 0) ? 2 : (r % 3 == 0) ? 3 : (r % 5 == 0) ? 5 : r;
}

template <int R, int S, class T>
struct Dft {
    static constexpr int A = first_factor(R);
    static constexpr int B = R / A;
    static_assert(A > 1 && B > 1, "radix must be a product of 2, 3, 5");
    static __device__ __forceinline__ void run(cpx<T> *v) {
        cpx<T> t[R];
        static_for<0, B>([&](auto I2) {
            constexpr int n2 = I2;
            cpx<T> u[A];
            static_for<0, A>([&](auto I1) { u[I1] = v[int(I1) * B + n2]; });
            Dft<A, S, T>::run(u);
            static_for<0, A>([&](auto K1) {
                constexpr int k1 = K1;
                t[k1 * B + n2] = twc<S, long(n2) * k1, R>(u[k1]);
            });
        });
        static_for<0, A>([&](auto K1) {
            constexpr int k1 = K1;
            cpx<T> u[B];
            static_for<0, B>([&](auto I2) { u[I2] = t[k1 * B + int(I2)]; });
            Dft<B, S, T>::run(u);
            static_for<0, B>([&](auto K2) { v[k1 + A * int(K2)] = u[K2]; });
        });
    }
};

template <int S, class T>
struct Dft<1, S, T> {
    static __device__ __forceinline__ void run(cpx<T> *) {}
};
template <int S, class T>
struct Dft<2, S, T> {
    static __device__ __forceinline__ void run(cpx<T> *v) {
        cpx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};
template <int S, class T>
struct Dft<3, S, T> {
    static __device__ __forceinline__ void run(cpx<T> *v) {
        constexpr T h = T(0.86602540378443864676372317075293618);   // sin(2 pi / 3)
        cpx<T> a = v[0], b = v[1], c = v[2];
        cpx<T> s = cadd(b, c);
        cpx<T> d = csub(b, c);
        cpx<T> m = {a.x - T(0.5) * s.x, a.y - T(0.5) * s.y};
        cpx<T> r = mul_si<S>(cscale(d, h));
        v[0] = cadd(a, s);
        v[1] = cadd(m, r);
        v[2] = csub(m, r);
    }
};
template <int S, class T>
struct Dft<4, S, T> {
    static __device__ __forceinline__ void run(cpx<T> *v) {
        cpx<T> a = v[0], b = v[1], c = v[2], d = v[3];
        cpx<T> s0 = cadd(a, c), d0 = csub(a, c);
        cpx<T> s1 = cadd(b, d), d1 = mul_si<S>(csub(b, d));
        v[0] = cadd(s0, s1);
        v[2] = csub(s0, s1);
        v[1] = cadd(d0, d1);
        v[3] = csub(d0, d1);
    }
};
template <int S, class T>
struct Dft<5, S, T> {
    static __device__ __forceinline__ void run(cpx<T> *v) {
        constexpr T c1 = T(0.30901699437494742410229341718281906);    // cos(2 pi/5)
        constexpr T c2 = T(-0.80901699437494742410229341718281906);   // cos(4 pi/5)
        constexpr T s1 = T(0.95105651629515357211643933337938214);    // sin(2 pi/5)
        constexpr T s2 = T(0.58778525229247312916870595463907277);    // sin(4 pi/5)
        cpx<T> a = v[0];
        cpx<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
        cpx<T> t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
        cpx<T> p1 = {a.x + c1 * t1.x + c2 * t2.x, a.y + c1 * t1.y + c2 * t2.y};
        cpx<T> p2 = {a.x + c2 * t1.x + c1 * t2.x, a.y + c2 * t1.y + c1 * t2.y};
        cpx<T> q1 = mul_si<S>(cpx<T>{s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y});
        cpx<T> q2 = mul_si<S>(cpx<T>{s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y});
        v[0] = cadd(a, cadd(t1, t2));
        v[1] = cadd(p1, q1);
        v[4] = csub(p1, q1);
        v[2] = cadd(p2, q2);
        v[3] = csub(p2, q2);
    }
};

// ---- factorisation of N into R1 * R2 ----------------------------------------
constexpr bool smooth(int r) {
    while (r % 2 == 0) r /= 2;
    while (r % 3 == 0) r /= 3;
    while (r % 5 == 0) r /= 5;
    return r == 1;
}
constexpr int isqrt(int n) {
    int r = 0;
    while ((r + 1) * (r + 1) <= n) ++r;
    return r;
}
// Default split: a first-stage radix R1 = 8 where it fits (measured fastest for
// the plane pass at N = 72, 96 and 120), else the largest R2 <= sqrt(N).
constexpr int choose_r2(int n) {
    if (n % 8 == 0 && n / 8 >= 2 && n / 8 <= 16 && smooth(n / 8)) return n / 8;
    for (int r2 = isqrt(n); r2 >= 1; --r2)
        if (n % r2 == 0 && n / r2 <= 16 && smooth(r2) && smooth(n / r2)) return r2;
    return 0;
}
// N = R1 * R2 with both factors in [2, 16] and products of 2, 3, 5: the
// alternative radix splits a context may be tuned to (choose_r2 is the default)
constexpr bool split_ok(int n, int r2) {
    return r2 >= 2 && r2 <= 16 && n % r2 == 0 && n / r2 >= 2 && n / r2 <= 16 && smooth(r2) &&
           smooth(n / r2);
}
template <int N_, int R2_ = 0>
struct Split {
    static constexpr int N = N_;
    static constexpr int R2 = R2_ > 0 ? R2_ : choose_r2(N_);
    static constexpr int R1 = N_ / R2;
    static_assert(R2 > 0 && R2 <= 16 && R1 <= 16 && R1 * R2 == N_, "unsupported FFT length or split");
};

// Position of frequency k in a dit result.
template <class P>
__device__ __forceinline__ int digit_rev(int k) {
    return (k % P::R1) * P::R2 + k / P::R1;
}
// Frequency held at position p of a dit result.
template <class P>
__device__ __forceinline__ int freq_at(int p) {
    return (p / P::R2) + P::R1 * (p % P::R2);
}

template <int S, class T>
__device__ __forceinline__ cpx<T> twiddle(const cpx<T> *tw, int idx) {
    cpx<T> w = tw[idx];
    if constexpr (S < 0) w.y = -w.y;
    return w;
}

// dit stage A of item n2 on its R1 inputs u[n1] = x[n1 R2 + n2], in registers:
// leaves the value for position k1 R2 + n2 in u[k1].
template <class P, int S, class T>
__device__ __forceinline__ void dit_a_regs(cpx<T> *u, int n2, const cpx<T> *tw) {
    constexpr int N = P::N, R1 = P::R1;
    Dft<R1, S, T>::run(u);
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1) u[k1] = cmul(u[k1], twiddle<S>(tw, (n2 * k1) % N));
}
// dit stage A on one sequence (element stride 1): item n2 in [0, R2).
template <class P, int S, class T>
__device__ __forceinline__ void dit_a(cpx<T> *x, int n2, const cpx<T> *tw) {
    constexpr int R1 = P::R1, R2 = P::R2;
    cpx<T> u[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) u[n1] = x[n1 * R2 + n2];
    dit_a_regs<P, S>(u, n2, tw);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) x[k1 * R2 + n2] = u[k1];
}
// dit stage B: item k1 in [0, R1); leaves X[k1 + R1 k2] in out[k2].
template <class P, int S, class T>
__device__ __forceinline__ void dit_b(const cpx<T> *x, int k1, cpx<T> *out) {
    constexpr int R2 = P::R2;
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) out[n2] = x[k1 * R2 + n2];
    Dft<R2, S, T>::run(out);
}
// dif stage B': item k1 in [0, R1), in place.
template <class P, int S, class T>
__device__ __forceinline__ void dif_b(cpx<T> *x, int k1) {
    constexpr int R2 = P::R2;
    cpx<T> u[R2];
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) u[k2] = x[k1 * R2 + k2];
    Dft<R2, S, T>::run(u);
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) x[k1 * R2 + n2] = u[n2];
}
// dif stage A': item n2 in [0, R2); leaves x[n1 R2 + n2] in out[n1].
template <class P, int S, class T>
__device__ __forceinline__ void dif_a(const cpx<T> *x, int n2, const cpx<T> *tw, cpx<T> *out) {
    constexpr int N = P::N, R1 = P::R1, R2 = P::R2;
    out[0] = x[n2];
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1) out[k1] = cmul(x[k1 * R2 + n2], twiddle<S>(tw, (n2 * k1) % N));
    Dft<R1, S, T>::run(out);
}

}  // namespace fft
}  // namespace pw
