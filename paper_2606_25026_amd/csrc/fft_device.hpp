// Device-side FFT building blocks for gfx950: complex arithmetic, radix-2/3/4
// butterflies composed into radices 6/8/12/16/24 with compile-time twiddle
// constants, and a multi-level Stockham pencil FFT whose levels exchange data
// through LDS.  A pencil of length N is held by T cooperating lanes, E = N/T
// complex values per lane; each level applies E/R radix-R butterflies per lane.
//
// Transform convention: forward X[k] = sum_n x[n] exp(-2 pi i n k / N),
// inverse with exp(+2 pi i n k / N), both unnormalised (the 1/N factors of the
// split step are folded into the phase and Green's-function multiplies).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

namespace wdm {

template <typename R>
struct cplx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cplx<R> operator+(cplx<R> a, cplx<R> b) {
    return {a.re + b.re, a.im + b.im};
}
template <typename R>
__device__ __forceinline__ cplx<R> operator-(cplx<R> a, cplx<R> b) {
    return {a.re - b.re, a.im - b.im};
}
template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename R>
__device__ __forceinline__ cplx<R> cmulc(cplx<R> a, cplx<R> b) {
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename R>
__device__ __forceinline__ cplx<R> cscale(cplx<R> a, R s) {
    return {a.re * s, a.im * s};
}
template <typename R>
__device__ __forceinline__ cplx<R> conj(cplx<R> a) {
    return {a.re, -a.im};
}
// a * (h + l) for a twiddle split into a high part h and a small low part l,
// rounded once per component: the low terms enter the fused chain before the
// single rounding of the large product.  (Adding a*l after rounding a*h would
// round the correction away and leave the constant's modulus error in place,
// which biases the norm by ~1e-8 per butterfly in the same direction every
// step.)
template <typename R>
__device__ __forceinline__ cplx<R> cmul_split(cplx<R> a, cplx<R> h, cplx<R> l) {
    R re = fma(a.re, l.re, -(a.im * l.im));
    re = fma(-a.im, h.im, re);
    re = fma(a.re, h.re, re);
    R im = fma(a.re, l.im, a.im * l.re);
    im = fma(a.im, h.re, im);
    im = fma(a.re, h.im, im);
    return {re, im};
}

// multiply by -i (forward direction) or +i (inverse direction)
template <bool INV, typename R>
__device__ __forceinline__ cplx<R> mul_mi(cplx<R> a) {
    if constexpr (INV)
        return {-a.im, a.re};
    else
        return {a.im, -a.re};
}

// Global-memory complex load / store through 2-vectors of the base type
// (address space 1, see wdm_internal.hpp).
typedef float wdm_f2v __attribute__((ext_vector_type(2)));
typedef double wdm_d2v __attribute__((ext_vector_type(2)));
template <typename T>
struct Vec2;
template <>
struct Vec2<float> {
    using type = wdm_f2v;
};
template <>
struct Vec2<double> {
    using type = wdm_d2v;
};
template <typename T>
__device__ __forceinline__ cplx<T> gld(const cplx<T>* p, int64_t i) {
    using V = typename Vec2<T>::type;
    const V v = ((const __attribute__((address_space(1))) V*)p)[i];
    return {v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void gst(cplx<T>* p, int64_t i, cplx<T> v) {
    using V = typename Vec2<T>::type;
    ((__attribute__((address_space(1))) V*)p)[i] = V{v.re, v.im};
}

// ---------------------------------------------------------------------------
// compile-time helpers
// ---------------------------------------------------------------------------
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// cos(2 pi j / 48) on the first quadrant; exact symmetric values elsewhere.
constexpr double kQuarterCos48[13] = {
    1.0,
    0.99144486137381041114,
    0.96592582628906828675,
    0.92387953251128675613,
    0.86602540378443864676,
    0.79335334029123516458,
    0.70710678118654752440,
    0.60876142900872063942,
    0.5,
    0.38268343236508977173,
    0.25881904510252076235,
    0.13052619222005159155,
    0.0};

constexpr double cos48(int j) {
    j = ((j % 48) + 48) % 48;
    if (j <= 12) return kQuarterCos48[j];
    if (j <= 24) return -kQuarterCos48[24 - j];
    if (j <= 36) return -kQuarterCos48[j - 24];
    return kQuarterCos48[48 - j];
}
constexpr double sin48(int j) { return cos48(j - 12); }

// a * W_R^E with W_R = exp(-2 pi i / R) (forward) or its conjugate (inverse).
// R must divide 48.  In single precision the constant is carried as a
// hi + lo pair of floats: a rounded constant has a fixed modulus error
// (|w|^2 - 1 = -5.7e-8 for 22.5 degrees), which would bias the norm the same
// way in every butterfly of every step; with the pair the product is exact up
// to one rounding of the result.
template <int R, int E, bool INV, typename T>
__device__ __forceinline__ cplx<T> twiddle_const(cplx<T> a) {
    static_assert(48 % R == 0, "radix must divide 48");
    constexpr int j = ((E % R) * (48 / R)) % 48;
    if constexpr (j == 0) {
        return a;
    } else if constexpr (j == 24) {
        return {-a.re, -a.im};
    } else if constexpr (j == 12) {
        return mul_mi<INV>(a);                 // W = -i (forward)
    } else if constexpr (j == 36) {
        return mul_mi<!INV>(a);                // W = +i (forward)
    } else {
        constexpr double cd = cos48(j);
        constexpr double sd = INV ? sin48(j) : -sin48(j);
        constexpr T c = T(cd);
        constexpr T s = T(sd);
        if constexpr (std::is_same<T, float>::value) {
            constexpr float cl = float(cd - double(c));
            constexpr float sl = float(sd - double(s));
            return cmul_split(a, cplx<T>{c, s}, cplx<T>{cl, sl});
        } else {
            return cplx<T>{a.re * c - a.im * s, a.re * s + a.im * c};
        }
    }
}

template <int R>
constexpr int first_factor() {
    if (R % 4 == 0 && R > 4) return 4;
    if (R % 2 == 0 && R > 2) return 2;
    if (R % 3 == 0 && R > 3) return 3;
    return R;
}

// In-register DFT of length R (natural order in, natural order out).
template <int R, bool INV, typename T>
__device__ __forceinline__ void dft(cplx<T>* v) {
    if constexpr (R == 1) {
        return;
    } else if constexpr (R == 2) {
        cplx<T> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    } else if constexpr (R == 3) {
        // X1,2 = x0 - (x1+x2)/2 -/+ i (sqrt3/2)(x1 - x2)  (forward)
        constexpr double hd = 0.86602540378443864676;
        constexpr T h = T(hd);
        cplx<T> s = v[1] + v[2];
        cplx<T> d = v[1] - v[2];
        cplx<T> m = {v[0].re - T(0.5) * s.re, v[0].im - T(0.5) * s.im};
        cplx<T> hd_ = {d.re * h, d.im * h};
        if constexpr (std::is_same<T, float>::value) {
            constexpr float hl = float(hd - double(h));   // low half of sqrt(3)/2
            hd_ = cplx<T>{fma(d.re, h, d.re * hl), fma(d.im, h, d.im * hl)};
        }
        cplx<T> r = mul_mi<INV>(hd_);
        v[0] = v[0] + s;
        v[1] = m + r;
        v[2] = m - r;
    } else if constexpr (R == 4) {
        cplx<T> a = v[0] + v[2], b = v[0] - v[2];
        cplx<T> c = v[1] + v[3], d = mul_mi<INV>(v[1] - v[3]);
        v[0] = a + c;
        v[2] = a - c;
        v[1] = b + d;
        v[3] = b - d;
    } else {
        // R = A * B: n = B n1 + n2, k = k1 + A k2
        constexpr int A = first_factor<R>();
        constexpr int B = R / A;
        cplx<T> tmp[R];
        static_for<0, B>([&](auto n2c) {
            constexpr int n2 = decltype(n2c)::value;
            cplx<T> u[A];
            static_for<0, A>([&](auto n1c) {
                constexpr int n1 = decltype(n1c)::value;
                u[n1] = v[B * n1 + n2];
            });
            dft<A, INV, T>(u);
            static_for<0, A>([&](auto k1c) {
                constexpr int k1 = decltype(k1c)::value;
                tmp[n2 * A + k1] = twiddle_const<R, n2 * k1, INV>(u[k1]);
            });
        });
        static_for<0, A>([&](auto k1c) {
            constexpr int k1 = decltype(k1c)::value;
            cplx<T> u[B];
            static_for<0, B>([&](auto n2c) {
                constexpr int n2 = decltype(n2c)::value;
                u[n2] = tmp[n2 * A + k1];
            });
            dft<B, INV, T>(u);
            static_for<0, B>([&](auto k2c) {
                constexpr int k2 = decltype(k2c)::value;
                v[k1 + A * k2] = u[k2];
            });
        });
    }
}

// ---------------------------------------------------------------------------
// Stockham plan: N = R0 * R1 * ... ; T lanes per pencil, E = N / T per lane.
// ---------------------------------------------------------------------------
template <int N_, int T_, int... Rs>
struct FftPlan {
    static constexpr int N = N_;
    static constexpr int T = T_;
    static constexpr int E = N_ / T_;
    static constexpr int L = sizeof...(Rs);
    static constexpr int radix[L] = {Rs...};
    static constexpr int stride_before(int l) {
        int s = 1;
        for (int i = 0; i < l; ++i) s *= radix[i];
        return s;
    }
    static constexpr int first() { return radix[0]; }
    static constexpr int last() { return radix[L - 1]; }
    static constexpr bool valid() {
        if (stride_before(L) != N || E * T != N) return false;
        for (int i = 0; i < L; ++i)
            if (E % radix[i] != 0 || 48 % radix[i] != 0) return false;
        return true;
    }
};

// Reversed plan, used for the inverse transform so that its input layout is
// the forward transform's output layout.
template <class P, class Seq>
struct ReverseHelper;
template <class P, std::size_t... I>
struct ReverseHelper<P, std::index_sequence<I...>> {
    using type = FftPlan<P::N, P::T, P::radix[P::L - 1 - I]...>;
};
// The same plan with twice the pencils per work-group of the strided passes
// (256-byte row segments for complex64): an autotuner choice.
template <class P>
struct WideRows : P {
    static constexpr int kRowMul = 2;
};
template <class Q, std::size_t... I>
struct ReverseHelper<WideRows<Q>, std::index_sequence<I...>> {
    using type = WideRows<typename ReverseHelper<Q, std::index_sequence<I...>>::type>;
};
// The same plan exchanging whole complex values through LDS (one barrier pair
// per level instead of two, twice the LDS) where the default splits real and
// imaginary parts: an autotuner choice.
template <class P>
struct ComplexExchange : P {
    static constexpr bool kComplexX = true;
};
template <class Q, std::size_t... I>
struct ReverseHelper<ComplexExchange<Q>, std::index_sequence<I...>> {
    using type = ComplexExchange<typename ReverseHelper<Q, std::index_sequence<I...>>::type>;
};
template <class P>
using Reversed = typename ReverseHelper<P, std::make_index_sequence<P::L>>::type;

// Register slot s = b * R + r of lane t holds pencil element t + T b + r N / R,
// where R is the first radix (input layout) or the last radix (output layout).
template <class P, int R>
__device__ __forceinline__ constexpr int slot_elem_c(int t, int s) {
    return t + P::T * (s / R) + (s % R) * (P::N / R);
}

// One Stockham level (LVL) applied to the lane's registers.  `lds(e)` maps a
// pencil element to this pencil's LDS slot; `tw` is W_N^m, m in [0, N), in LDS.
// Levels > 0 read their inputs from LDS; all levels but the last write their
// outputs to LDS.  Callers guarantee the LDS region is free on entry.
template <class P, int LVL, bool INV, typename T, class Idx>
__device__ __forceinline__ void stockham_level(cplx<T>* v, cplx<T>* lds, const cplx<T>* tw,
                                               int t, Idx idx) {
    constexpr int R = P::radix[LVL];
    constexpr int Ns = P::stride_before(LVL);
    constexpr int NB = P::E / R;
    constexpr int N = P::N;
    if constexpr (LVL > 0) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = t + P::T * b;
#pragma unroll
            for (int r = 0; r < R; ++r) v[b * R + r] = lds[idx(j + r * (N / R))];
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = t + P::T * b;
            const int jm = j % Ns;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const int m = jm * r * (N / (Ns * R));
                const cplx<T> x = v[b * R + r];
                if constexpr (std::is_same<T, float>::value) {
                    // hi (entries 0..N-1) and lo (N..2N-1) halves, one rounding
                    const cplx<T> h = tw[m], l = tw[N + m];
                    v[b * R + r] = INV ? cmul_split(x, conj(h), conj(l)) : cmul_split(x, h, l);
                } else {
                    v[b * R + r] = INV ? cmulc(x, tw[m]) : cmul(x, tw[m]);
                }
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) dft<R, INV, T>(v + b * R);
    if constexpr (LVL + 1 < P::L) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = t + P::T * b;
            const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
            for (int r = 0; r < R; ++r) lds[idx(base + r * Ns)] = v[b * R + r];
        }
        __syncthreads();
        stockham_level<P, LVL + 1, INV, T>(v, lds, tw, t, idx);
    }
}

// stockham_level with the LDS exchange split in two: the real parts move
// through a buffer of one real value per pencil element, then the imaginary
// parts through the same buffer.  Half the LDS of the complex exchange, for
// two more barriers per level; a lane's imaginary parts stay in its registers
// while the real parts are exchanged.
template <class P, int LVL, bool INV, typename T, class Idx>
__device__ __forceinline__ void stockham_level_split(cplx<T>* v, T* lds, const cplx<T>* tw,
                                                     int t, Idx idx) {
    constexpr int R = P::radix[LVL];
    constexpr int Ns = P::stride_before(LVL);
    constexpr int NB = P::E / R;
    constexpr int N = P::N;
    if constexpr (LVL > 0) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = t + P::T * b;
            const int jm = j % Ns;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const int m = jm * r * (N / (Ns * R));
                const cplx<T> x = v[b * R + r];
                if constexpr (std::is_same<T, float>::value) {
                    const cplx<T> h = tw[m], l = tw[N + m];
                    v[b * R + r] = INV ? cmul_split(x, conj(h), conj(l)) : cmul_split(x, h, l);
                } else {
                    v[b * R + r] = INV ? cmulc(x, tw[m]) : cmul(x, tw[m]);
                }
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) dft<R, INV, T>(v + b * R);
    if constexpr (LVL + 1 < P::L) {
        constexpr int R2 = P::radix[LVL + 1];
        constexpr int NB2 = P::E / R2;
#pragma unroll
        for (int part = 0; part < 2; ++part) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int j = t + P::T * b;
                const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
                for (int r = 0; r < R; ++r)
                    lds[idx(base + r * Ns)] = part ? v[b * R + r].im : v[b * R + r].re;
            }
            __syncthreads();
#pragma unroll
            for (int b = 0; b < NB2; ++b) {
                const int j = t + P::T * b;
#pragma unroll
                for (int r = 0; r < R2; ++r) {
                    const T x = lds[idx(j + r * (N / R2))];
                    if (part)
                        v[b * R2 + r].im = x;
                    else
                        v[b * R2 + r].re = x;
                }
            }
            __syncthreads();
        }
        stockham_level_split<P, LVL + 1, INV, T>(v, lds, tw, t, idx);
    }
}

// Twiddle entries per table: complex64 keeps W_N^m as hi (first N entries) and
// lo (next N) floats; complex128 keeps one double table.
template <typename T>
constexpr int tw_entries(int n) {
    return std::is_same<T, float>::value ? 2 * n : n;
}

// Full pencil transform.  Input in the plan's input layout (first radix),
// output in its output layout (last radix).  Ends with no LDS reads pending
// only after the caller's next barrier.
template <class P, bool INV, typename T, class Idx>
__device__ __forceinline__ void pencil_fft(cplx<T>* v, cplx<T>* lds, const cplx<T>* tw, int t,
                                           Idx idx) {
    static_assert(P::valid(), "invalid FFT plan");
    stockham_level<P, 0, INV, T>(v, lds, tw, t, idx);
}

// The same transform with the split exchange (one real LDS value per pencil
// element).  Ends with every LDS read done (the last exchange's barrier).
template <class P, bool INV, typename T, class Idx>
__device__ __forceinline__ void pencil_fft(cplx<T>* v, T* lds, const cplx<T>* tw, int t,
                                           Idx idx) {
    static_assert(P::valid(), "invalid FFT plan");
    stockham_level_split<P, 0, INV, T>(v, lds, tw, t, idx);
}

}  // namespace wdm
