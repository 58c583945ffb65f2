// Shared pieces of the grid passes of the kick-drift-kick split step
// (Sec. 3.1, Eq. SPE_solver_KDK; Sec. 3.2.1 for the periodic Poisson solve):
// FFT plans per axis length, lane/LDS mappings of pencils, slot loads and
// stores, the kick rotation, the kinetic factor tables and launch helpers.
// The passes themselves live in passes_z.hip (P1, P5), passes_y.hip (P2, P4,
// P6, P8) and passes_x.hip (P3, P7).  Each pass streams one 3D array once
// through HBM: a work-group owns P pencils of one axis, loads them with
// 128-byte row segments, transforms them in registers + LDS and fuses the
// pointwise work of the method into the same pass:
//
//   P1  z: half spectrum -> Phi (C2R), kick psi by exp(-i Phi tau/eta), z-FFT
//   P2  y: forward FFT of psi
//   P3  x: forward FFT, kinetic phase exp(-i eta |k|^2 dt / 2) / N, inverse FFT
//   P4  y: inverse FFT of psi
//   P5  z: inverse FFT of psi, rho = |psi|^2 + rho_b (rho_b cleared), R2C z-FFT
//   P6  y: forward FFT of the half spectrum (+ the kz = nz/2 plane)
//   P7  x: forward FFT, Green's function -4 pi G / |k|^2 / N, inverse FFT
//   P8  y: inverse FFT of the half spectrum
//
// Phase arguments (Phi tau / eta and eta |k|^2 dt / 2) are formed in FP64 and
// reduced mod 2 pi; the kinetic factors are FP64-formed tables.
#pragma once
#include "wdm_internal.hpp"
#include "fft_device.hpp"

namespace wdm {

// ---------------------------------------------------------------------------
// FFT schedule per axis length: Stockham radices and lanes per pencil.  V = 0
// is the default plan; V = 1 (where listed) uses twice the lanes per pencil and
// half the values per lane (one more LDS exchange, half the registers), a
// choice the plan's autotuner makes per pass by timing both.
// ---------------------------------------------------------------------------
template <int N, int V = 0>
struct PlanFor;
template <> struct PlanFor<16, 0> { using type = FftPlan<16, 4, 4, 4>; };
template <> struct PlanFor<32, 0> { using type = FftPlan<32, 4, 8, 4>; };
template <> struct PlanFor<64, 0> { using type = FftPlan<64, 8, 8, 8>; };
template <> struct PlanFor<96, 0> { using type = FftPlan<96, 8, 4, 6, 4>; };
template <> struct PlanFor<128, 0> { using type = FftPlan<128, 8, 16, 8>; };
template <> struct PlanFor<192, 0> { using type = FftPlan<192, 16, 4, 12, 4>; };
template <> struct PlanFor<256, 0> { using type = FftPlan<256, 16, 16, 16>; };
template <> struct PlanFor<384, 0> { using type = FftPlan<384, 16, 8, 6, 8>; };
template <> struct PlanFor<512, 0> { using type = FftPlan<512, 32, 8, 4, 16>; };
template <> struct PlanFor<32, 1> { using type = FftPlan<32, 8, 4, 4, 2>; };
template <> struct PlanFor<64, 1> { using type = FftPlan<64, 16, 4, 4, 4>; };
template <> struct PlanFor<128, 1> { using type = FftPlan<128, 16, 8, 4, 4>; };
template <> struct PlanFor<256, 1> { using type = FftPlan<256, 32, 8, 8, 4>; };
template <> struct PlanFor<384, 1> { using type = FftPlan<384, 32, 6, 4, 4, 4>; };
template <> struct PlanFor<512, 1> { using type = FftPlan<512, 64, 8, 8, 8>; };

// V = 2 (strided passes only): the default radices with twice the pencils per
// work-group (row segments of 256 bytes for complex64), for lengths up to 256.
template <int N>
struct PlanFor<N, 2> {
    using type = WideRows<typename PlanFor<N, 0>::type>;
};

// V = 3: the default radices with the complex LDS exchange -- the strided
// passes at lengths up to 256 (has_wide), the z passes at the lengths whose
// default splits the exchange (has_zcx).
template <int N>
struct PlanFor<N, 3> {
    using type = ComplexExchange<typename PlanFor<N, 0>::type>;
};

// Lengths with a second plan.
constexpr bool has_variant(int n) {
    return n == 32 || n == 64 || n == 128 || n == 256 || n == 384 || n == 512;
}
// Lengths with the wide-row and complex-exchange plans of the strided passes.
constexpr bool has_wide(int n) {
    return n == 16 || n == 32 || n == 64 || n == 96 || n == 128 || n == 192 || n == 256;
}
static_assert(PlanFor<16>::type::valid() && PlanFor<32>::type::valid() &&
                  PlanFor<64>::type::valid() && PlanFor<96>::type::valid() &&
                  PlanFor<128>::type::valid() && PlanFor<192>::type::valid() &&
                  PlanFor<256>::type::valid() && PlanFor<384>::type::valid() &&
                  PlanFor<512>::type::valid(),
              "default plans");
static_assert(PlanFor<32, 1>::type::valid() && PlanFor<64, 1>::type::valid() &&
                  PlanFor<128, 1>::type::valid() && PlanFor<256, 1>::type::valid() &&
                  PlanFor<384, 1>::type::valid() && PlanFor<512, 1>::type::valid(),
              "second plans");

// Row-segment multiplier of a plan (2 for WideRows).
template <class P, class = void>
struct RowMul {
    static constexpr int v = 1;
};
template <class P>
struct RowMul<P, std::void_t<decltype(P::kRowMul)>> {
    static constexpr int v = P::kRowMul;
};

// Pencils per work-group: at least 128 bytes per row segment (256 for a
// wide-row plan), at least 256 lanes.
template <class P, typename T>
constexpr int pencils_per_wg() {
    constexpr int pmin = 128 * RowMul<P>::v / int(sizeof(cplx<T>));
    constexpr int pfill = 256 / P::T;
    return pmin > pfill ? pmin : pfill;
}
template <class P, typename T>
constexpr int wg_size() {
    return pencils_per_wg<P, T>() * P::T;
}
template <class P, typename T, bool STRIDED>
constexpr int lds_entries() {
    // strided layout: N * PP entries; contiguous layout: PP * (N + N/16).  The
    // passes exchange real and imaginary parts in turn, one real per entry.
    return pencils_per_wg<P, T>() * (STRIDED ? P::N : P::N + P::N / 16);
}

// Whether a pass exchanges real and imaginary parts in turn (one real LDS
// entry per element) or whole complex values.  The split halves the LDS and,
// for the strided passes and the two-level plans, also lowers the register
// count; along the contiguous axis the three-level plans (96, 192, 384, 512)
// need more registers with it (P1 at 512: 114 -> 131, 3 waves per SIMD, 628
// -> 1125 us a pass), so they keep the complex exchange.
// A ComplexExchange plan always exchanges whole complex values.
template <class P, class = void>
struct IsComplexX {
    static constexpr bool v = false;
};
template <class P>
struct IsComplexX<P, std::void_t<decltype(P::kComplexX)>> {
    static constexpr bool v = P::kComplexX;
};
template <class P, bool STRIDED>
constexpr bool split_exchange() {
    return !IsComplexX<P>::v && (STRIDED || P::L <= 2);
}
template <class P, typename T, bool STRIDED>
using lds_t = std::conditional_t<split_exchange<P, STRIDED>(), T, cplx<T>>;
// Lengths whose contiguous-axis (z) passes split the exchange by default (the
// two-level plans), so that the complex-exchange plan differs for them too.
constexpr bool has_zcx(int n) {
    return n == 16 || n == 32 || n == 64 || n == 128 || n == 256;
}
static_assert(split_exchange<PlanFor<16>::type, false>() &&
                  split_exchange<PlanFor<32>::type, false>() &&
                  split_exchange<PlanFor<64>::type, false>() &&
                  split_exchange<PlanFor<128>::type, false>() &&
                  split_exchange<PlanFor<256>::type, false>() &&
                  !split_exchange<PlanFor<96>::type, false>() &&
                  !split_exchange<PlanFor<512>::type, false>(),
              "z-pass lengths with a complex-exchange plan");
// LDS element type of the strided-axis passes (whose Nyquist-plane tiles use
// the contiguous mapping with the same exchange).
template <class P, typename T>
using strided_lds_t = std::conditional_t<IsComplexX<P>::v, cplx<T>, T>;

// Lane coordinates and LDS addressing for the two pencil mappings.
//   strided:    neighbouring lanes take neighbouring pencils (rows in memory
//               run across pencils), LDS slot e * PP + p
//   contiguous: neighbouring lanes take neighbouring elements of one pencil,
//               LDS slot p * (N + N/16) + e + e/16 (skewed against conflicts)
template <class P, typename T, bool STRIDED>
struct Lanes {
    static constexpr int PP = pencils_per_wg<P, T>();
    int t, p;
    __device__ __forceinline__ Lanes() {
        const int tid = int(threadIdx.x);
        if constexpr (STRIDED) {
            p = tid % PP;
            t = tid / PP;
        } else {
            t = tid % P::T;
            p = tid / P::T;
        }
    }
    __device__ __forceinline__ int operator()(int e) const {
        if constexpr (STRIDED)
            return e * PP + p;
        else
            return p * (P::N + P::N / 16) + e + (e >> 4);
    }
};

template <class P, int R>
__device__ __forceinline__ int slot_elem(int t, int s) {
    return t + P::T * (s / R) + (s % R) * (P::N / R);
}

// Twiddle table of an N-point plan into LDS by a work-group of WG lanes.  The
// trip count is a compile-time constant so that every load is issued before
// the first wait.
template <int N, int WG, typename T>
__device__ __forceinline__ void load_twiddles(cplx<T>* tw, const void* g) {
    const cplx<T>* src = static_cast<const cplx<T>*>(g);
    constexpr int total = tw_entries<T>(N);
    constexpr int iters = (total + WG - 1) / WG;
    cplx<T> r[iters];
#pragma unroll
    for (int k = 0; k < iters; ++k) {
        const int i = int(threadIdx.x) + k * WG;
        r[k] = (total % WG == 0 || i < total) ? gld(src, i) : cplx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int k = 0; k < iters; ++k) {
        const int i = int(threadIdx.x) + k * WG;
        if (total % WG == 0 || i < total) tw[i] = r[k];
    }
}

__device__ __forceinline__ int signed_mode(int i, int n) { return i < n / 2 ? i : i - n; }

// Large-argument branch of rotate(): FP64 sincos and product, rounded once.
// Kept out of line: it is rarely taken and would otherwise be inlined into
// every slot of every pass.
// A non-finite argument (a non-finite potential, which the stability watch
// reports) rotates by zero rather than reaching sincos.
__device__ __noinline__ cplx<float> rotate_fp64(cplx<float> a, double r) {
    double s, c;
    sincos(__builtin_isfinite(r) ? r : 0.0, &s, &c);
    const double re = double(a.re), im = double(a.im);
    return cplx<float>{float(re * c - im * s), float(re * s + im * c)};
}

// a * exp(i arg), arg reduced mod 2 pi in FP64.  Single precision: for small
// reduced arguments exp(i r) = 1 + q with q = (cos r - 1, sin r) from their
// Taylor series (|r| < 1/16: the first omitted terms are below 1e-13 of the
// kept ones), so the factor's rounding error scales with |r| instead of sitting
// at the unit-modulus level; larger arguments take FP64 sincos and an FP64
// product, rounded once.
template <typename T>
__device__ __forceinline__ cplx<T> rotate(cplx<T> a, double arg) {
    const double r = arg - kTwoPi * rint(arg * (1.0 / kTwoPi));
    if constexpr (std::is_same<T, float>::value) {
        if (fabs(r) < 0.0625) {
            const float x = float(r), x2 = x * x;
            // cos x - 1 = -x^2/2! + x^4/4! - x^6/6! + x^8/8!
            const float qr =
                x2 * fmaf(x2, fmaf(x2, fmaf(x2, 1.0f / 40320.0f, -1.0f / 720.0f), 1.0f / 24.0f),
                          -0.5f);
            // sin x = x - x^3/3! + x^5/5! - x^7/7!
            const float qi =
                x * fmaf(x2, fmaf(x2, fmaf(x2, -1.0f / 5040.0f, 1.0f / 120.0f), -1.0f / 6.0f),
                         1.0f);
            // a (1 + q), fused so the small rotation is not rounded twice
            return cplx<float>{fma(a.re, qr, fma(-a.im, qi, a.re)),
                               fma(a.im, qr, fma(a.re, qi, a.im))};
        }
        return rotate_fp64(a, r);
    } else {
        double s, c;
        sincos(__builtin_isfinite(r) ? r : 0.0, &s, &c);
        return cmul(a, cplx<double>{c, s});
    }
}

// exp(i arg) in FP64 (argument reduced mod 2 pi first).
__device__ __forceinline__ cplx<double> expi64(double arg) {
    const double r = arg - kTwoPi * rint(arg * (1.0 / kTwoPi));
    double s, c;
    sincos(r, &s, &c);
    return cplx<double>{c, s};
}

// a * f with an FP64 factor, rounded once to T.
template <typename T>
__device__ __forceinline__ cplx<T> mul64(cplx<T> a, cplx<double> f) {
    const double re = double(a.re), im = double(a.im);
    return cplx<T>{T(re * f.re - im * f.im), T(re * f.im + im * f.re)};
}

// Generic load / store of the lane's slots of pencil `base`, element stride
// `st`.  Element slot_elem(t, s) = t + c_s with a compile-time c_s, so the
// lane's address is formed once and each slot adds the uniform c_s * st.
template <class P, int R>
__device__ __forceinline__ constexpr int slot_const(int s) {
    return P::T * (s / R) + (s % R) * (P::N / R);
}
template <class P, int R, typename T, class L>
__device__ __forceinline__ void load_slots(cplx<T>* v, const cplx<T>* g, int64_t base,
                                           int64_t st, bool ok, const L& ln) {
    const cplx<T>* lane = g + (base + int64_t(ln.t) * st);
#pragma unroll
    for (int s = 0; s < P::E; ++s)
        v[s] = ok ? gld(lane, int64_t(slot_const<P, R>(s)) * st) : cplx<T>{T(0), T(0)};
}
template <class P, int R, typename T, class L>
__device__ __forceinline__ void store_slots(const cplx<T>* v, cplx<T>* g, int64_t base,
                                            int64_t st, bool ok, const L& ln) {
    if (!ok) return;
    cplx<T>* lane = g + (base + int64_t(ln.t) * st);
#pragma unroll
    for (int s = 0; s < P::E; ++s) gst(lane, int64_t(slot_const<P, R>(s)) * st, v[s]);
}

// Kinetic factor tables of the drift exp(-i eta dt |k|^2 / 2) / N (Sec. 3.1),
// factored as e_x(k_x) e_yz(k_y, k_z) and formed in FP64: each mode gets the
// same factor every step, so a factor rounded to single precision would add up
// coherently over a run.  complex64 keeps each factor as an unevaluated sum
// hi + lo of two complex64 numbers.  Written once per wdm_step call, after the
// call's dt is set (grid-stride over nx + ny nz entries), read by P3.
template <typename T>
__device__ __forceinline__ void write_kinetic_table(const MemberDev& m, double dt, int64_t nthr,
                                                    int64_t gtid) {
    const int nx = m.nx, ny = m.ny, nz = m.nz;
    const int64_t total = int64_t(nx) + int64_t(ny) * nz;
    const double a = -0.5 * m.eta * dt;
    const double inv_n = 1.0 / (double(nx) * double(ny) * double(nz));
    for (int64_t t = gtid; t < total; t += nthr) {
        cplx<double> e;
        if (t < nx) {
            const double kx = (kTwoPi / m.lx) * signed_mode(int(t), nx);
            e = expi64(a * kx * kx);
        } else {
            const int64_t u = t - nx;
            const double ky = (kTwoPi / m.ly) * signed_mode(int(u / nz), ny);
            const double kz = (kTwoPi / m.lz) * signed_mode(int(u % nz), nz);
            e = expi64(a * (ky * ky + kz * kz));
            e = cplx<double>{e.re * inv_n, e.im * inv_n};
        }
        if constexpr (std::is_same<T, float>::value) {
            const cplx<float> h{float(e.re), float(e.im)};
            const cplx<float> l{float(e.re - double(h.re)), float(e.im - double(h.im))};
            cplx<float>* k = static_cast<cplx<float>*>(m.kin);
            gst(k, 2 * t, h);
            gst(k, 2 * t + 1, l);
        } else {
            gst(static_cast<cplx<double>*>(m.kin), t, e);
        }
    }
}

// ===========================================================================
// Strided-axis passes.  A pencil q starts at base(q) = (q / inner) * outer +
// q % inner and has element stride `st`.
// ===========================================================================
struct Strides {
    int64_t count, inner, outer, st;
    __device__ __forceinline__ int64_t base(int64_t q) const {
        return (q / inner) * outer + (q % inner);
    }
};

// Plain transform of one batch of pencils.
template <class P, typename T, bool INV, bool STRIDED, typename LT>
__device__ __forceinline__ void transform_tile(cplx<T>* data, const Strides& sd, int64_t tile,
                                               LT* lds, const cplx<T>* tw) {
    using LN = Lanes<P, T, STRIDED>;
    const LN ln;
    const int64_t q = tile * LN::PP + ln.p;
    const bool ok = q < sd.count;
    const int64_t b = ok ? sd.base(q) : 0;
    cplx<T> v[P::E];
    load_slots<P, P::first()>(v, data, b, sd.st, ok, ln);
    pencil_fft<P, INV, T>(v, lds, tw, ln.t, ln);
    store_slots<P, P::last()>(v, data, b, sd.st, ok, ln);
}


// ---------------------------------------------------------------------------
// Stability watch (Sec. 3.5): the largest |x| over a lane's E values, reduced
// over the wavefront (DPP) and folded into the wavefront's own slot of the
// member's watch array by an unsigned 64-bit atomic maximum of the FP64 bit
// pattern (the sign bit cleared, so a NaN orders above +inf and is kept).  No
// two wavefronts of a launch share a slot, so the atomics never contend.  All
// lanes of the wavefront must call it.
// ---------------------------------------------------------------------------
extern "C" __device__ __attribute__((const)) unsigned int __ockl_wfred_max_u32(unsigned int);
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_max_u64(
    unsigned long long);

__device__ __forceinline__ void watch_store(unsigned long long* slots, int64_t n,
                                            unsigned long long bits) {
    const int64_t w = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (__lane_id() == 0 && w < n) atomicMax(slots + w, bits);
}
template <int E>
__device__ __forceinline__ void watch_max(unsigned long long* slots, int64_t n, const float* x) {
    unsigned int u = 0;
#pragma unroll
    for (int s = 0; s < E; ++s) u = max(u, __float_as_uint(x[s]) & 0x7fffffffu);
    u = __ockl_wfred_max_u32(u);
    watch_store(slots, n, (unsigned long long)__double_as_longlong(double(__uint_as_float(u))));
}
template <int E>
__device__ __forceinline__ void watch_max(unsigned long long* slots, int64_t n, const double* x) {
    unsigned long long u = 0;
#pragma unroll
    for (int s = 0; s < E; ++s)
        u = max(u, (unsigned long long)__double_as_longlong(x[s]) & 0x7fffffffffffffffull);
    watch_store(slots, n, __ockl_wfred_max_u64(u));
}

// ---------------------------------------------------------------------------
// host-side helpers: dispatch on the axis length, grid and block shapes
// ---------------------------------------------------------------------------
template <template <int> class F, typename... A>
static hipError_t dispatch_n(int n, A&&... a) {
    switch (n) {
        case 16: return F<16>::run(a...);
        case 32: return F<32>::run(a...);
        case 64: return F<64>::run(a...);
        case 96: return F<96>::run(a...);
        case 128: return F<128>::run(a...);
        case 192: return F<192>::run(a...);
        case 256: return F<256>::run(a...);
        case 384: return F<384>::run(a...);
        case 512: return F<512>::run(a...);
        default: return hipErrorInvalidValue;
    }
}

template <int N, typename T, int V = 0>
static int64_t tiles(int64_t pencils) {
    using FP = typename PlanFor<N, V>::type;
    constexpr int PP = pencils_per_wg<FP, T>();
    return (pencils + PP - 1) / PP;
}
template <int N, typename T, int V = 0>
static dim3 block() {
    return dim3(wg_size<typename PlanFor<N, V>::type, T>());
}

}  // namespace wdm
