// Grid passes of the kick-drift-kick split step (Sec. 3.1, Eq. SPE_solver_KDK;
// Sec. 3.2.1 for the periodic Poisson solve).  Each pass streams one 3D array
// once through HBM: a work-group owns P pencils of one axis, loads them with
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
// Phase arguments (Phi tau / eta and eta |k|^2 dt / 2) and the Green's
// function are formed in FP64 and reduced mod 2 pi before the single-precision
// sincos of the complex64 path.
#include "wdm_internal.hpp"
#include "fft_device.hpp"

namespace wdm {

// ---------------------------------------------------------------------------
// FFT schedule per axis length: Stockham radices and lanes per pencil.
// ---------------------------------------------------------------------------
template <int N>
struct PlanFor;
template <> struct PlanFor<16> { using type = FftPlan<16, 4, 4, 4>; };
template <> struct PlanFor<32> { using type = FftPlan<32, 4, 8, 4>; };
template <> struct PlanFor<64> { using type = FftPlan<64, 8, 8, 8>; };
template <> struct PlanFor<96> { using type = FftPlan<96, 8, 4, 6, 4>; };
template <> struct PlanFor<128> { using type = FftPlan<128, 8, 16, 8>; };
template <> struct PlanFor<192> { using type = FftPlan<192, 16, 4, 12, 4>; };
template <> struct PlanFor<256> { using type = FftPlan<256, 16, 16, 16>; };
template <> struct PlanFor<384> { using type = FftPlan<384, 16, 8, 6, 8>; };
template <> struct PlanFor<512> { using type = FftPlan<512, 32, 8, 4, 16>; };

bool axis_supported(int n) {
    switch (n) {
        case 16: case 32: case 64: case 96: case 128: case 192: case 256: case 384: case 512:
            return true;
        default:
            return false;
    }
}

// Pencils per work-group: at least 128 bytes per row segment, at least 256 lanes.
template <class P, typename T>
constexpr int pencils_per_wg() {
    constexpr int pmin = 128 / int(sizeof(cplx<T>));
    constexpr int pfill = 256 / P::T;
    return pmin > pfill ? pmin : pfill;
}
template <class P, typename T>
constexpr int wg_size() {
    return pencils_per_wg<P, T>() * P::T;
}
template <class P, typename T, bool STRIDED>
constexpr int lds_entries() {
    // strided layout: N * PP entries; contiguous layout: PP * (N + N/16)
    return pencils_per_wg<P, T>() * (STRIDED ? P::N : P::N + P::N / 16);
}

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
__device__ __noinline__ cplx<float> rotate_fp64(cplx<float> a, double r) {
    double s, c;
    sincos(r, &s, &c);
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
        sincos(r, &s, &c);
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
// hi + lo of two complex64 numbers.  Written by the threads of P1's merged
// variant (grid-stride over nx + ny nz entries), read by P3 of the same step.
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
// P1: potential from the half spectrum, kick, optional forward z-FFT.
// ===========================================================================
template <int NZ, typename T, int OP, int KICK>
__global__ __launch_bounds__((wg_size<typename PlanFor<NZ>::type, T>())) void k_z_potential_kick(
    const MemberDev* __restrict__ mems, int first) {
    using FP = typename PlanFor<NZ>::type;
    using IP = Reversed<FP>;
    using LN = Lanes<FP, T, false>;
    constexpr int PP = LN::PP;
    constexpr int H = NZ / 2;
    __shared__ cplx<T> lds[lds_entries<FP, T, false>()];
    __shared__ cplx<T> tw[tw_entries<T>(NZ)];
    const MemberDev& m = mems[first + blockIdx.y];
    const LN ln;
    const int64_t npen = int64_t(m.nx) * m.ny;
    const int64_t q = int64_t(blockIdx.x) * PP + ln.p;
    const bool ok = q < npen;
    load_twiddles<NZ, wg_size<FP, T>()>(tw, m.tw_z);
    // psi is loaded together with the spectrum: one memory wait per pass
    cplx<T>* psi = static_cast<cplx<T>*>(m.psi);
    cplx<T> w[OP == kZPhiOnly ? 1 : FP::E];
    if constexpr (OP != kZPhiOnly) load_slots<FP, FP::first()>(w, psi, q * NZ, 1, ok, ln);
    // half spectrum e in [0, H) (H / T per lane) and the Nyquist element e = H,
    // all loads issued before the LDS writes
    static_assert(H % FP::T == 0, "half pencil must split evenly over the lanes");
    constexpr int HE = H / FP::T;
    const cplx<T>* spec = static_cast<const cplx<T>*>(m.spec) + q * H + ln.t;
    cplx<T> hs[HE + 1];
#pragma unroll
    for (int k = 0; k < HE; ++k) hs[k] = ok ? gld(spec, k * FP::T) : cplx<T>{T(0), T(0)};
    hs[HE] = (ok && ln.t == 0) ? gld(static_cast<const cplx<T>*>(m.spec_nyq), q)
                               : cplx<T>{T(0), T(0)};
#pragma unroll
    for (int k = 0; k < HE; ++k) lds[ln(ln.t + k * FP::T)] = hs[k];
    if (ln.t == 0) lds[ln(H)] = hs[HE];
    __syncthreads();
    // Hermitian completion F[e] = conj(F[NZ - e]) for e > NZ/2, in the input
    // layout of the inverse plan
    cplx<T> v[FP::E];
#pragma unroll
    for (int s = 0; s < FP::E; ++s) {
        const int e = slot_elem<IP, IP::first()>(ln.t, s);
        v[s] = e <= H ? lds[ln(e)] : conj(lds[ln(NZ - e)]);
    }
    __syncthreads();
    pencil_fft<IP, true, T>(v, lds, tw, ln.t, ln);
    // output layout of IP == input layout of FP
    T phi[FP::E];
    T* gphi = static_cast<T*>(m.phi) + q * NZ;
#pragma unroll
    for (int s = 0; s < FP::E; ++s) {
        phi[s] = v[s].re;
        if (ok) gstr(gphi, slot_elem<FP, FP::first()>(ln.t, s), phi[s]);
    }
    if constexpr (OP == kZPhiOnly) return;
    const double dt = gldr(m.dt, 0);
    const double tau = (KICK == kFullKick) ? dt : 0.5 * dt;
    const double c = -tau / m.eta;
#pragma unroll
    for (int s = 0; s < FP::E; ++s) v[s] = rotate(w[s], double(phi[s]) * c);
    if constexpr (OP == kZKickOnly) {
        store_slots<FP, FP::first()>(v, psi, q * NZ, 1, ok, ln);
        return;
    }
    __syncthreads();
    pencil_fft<FP, false, T>(v, lds, tw, ln.t, ln);
    store_slots<FP, FP::last()>(v, psi, q * NZ, 1, ok, ln);
    write_kinetic_table<T>(m, dt, int64_t(gridDim.x) * blockDim.x,
                           int64_t(blockIdx.x) * blockDim.x + threadIdx.x);
}

// ===========================================================================
// P5: inverse z-FFT of psi, density, R2C forward z-FFT into the half spectrum.
// ===========================================================================
template <int NZ, typename T, int OP>
__global__ __launch_bounds__((wg_size<typename PlanFor<NZ>::type, T>())) void k_z_density(
    const MemberDev* __restrict__ mems, int first) {
    using FP = typename PlanFor<NZ>::type;
    using IP = Reversed<FP>;
    using LN = Lanes<FP, T, false>;
    constexpr int PP = LN::PP;
    constexpr int H = NZ / 2;
    __shared__ cplx<T> lds[lds_entries<FP, T, false>()];
    __shared__ cplx<T> tw[tw_entries<T>(NZ)];
    const MemberDev& m = mems[first + blockIdx.y];
    const LN ln;
    const int64_t npen = int64_t(m.nx) * m.ny;
    const int64_t q = int64_t(blockIdx.x) * PP + ln.p;
    const bool ok = q < npen;
    load_twiddles<NZ, wg_size<FP, T>()>(tw, m.tw_z);
    cplx<T>* psi = static_cast<cplx<T>*>(m.psi);
    cplx<T> v[FP::E];
    // the baryon density is loaded together with psi: one memory wait per pass
    T* rb = static_cast<T*>(m.rho_b) + q * NZ + ln.t;
    T rbv[FP::E];
#pragma unroll
    for (int s = 0; s < FP::E; ++s) rbv[s] = ok ? gldr(rb, slot_const<FP, FP::first()>(s)) : T(0);
    if constexpr (OP == kDensInvFft) {
        load_slots<IP, IP::first()>(v, psi, q * NZ, 1, ok, ln);
        __syncthreads();
        pencil_fft<IP, true, T>(v, lds, tw, ln.t, ln);
        store_slots<FP, FP::first()>(v, psi, q * NZ, 1, ok, ln);
    } else {
        load_slots<FP, FP::first()>(v, psi, q * NZ, 1, ok, ln);
        __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < FP::E; ++s) {
        v[s] = cplx<T>{v[s].re * v[s].re + v[s].im * v[s].im + rbv[s], T(0)};
        if (ok) gstr(rb, slot_const<FP, FP::first()>(s), T(0));
    }
    __syncthreads();
    pencil_fft<FP, false, T>(v, lds, tw, ln.t, ln);
    if (!ok) return;
    cplx<T>* spec = static_cast<cplx<T>*>(m.spec) + q * H;
#pragma unroll
    for (int s = 0; s < FP::E; ++s) {
        const int e = slot_elem<FP, FP::last()>(ln.t, s);
        if (e < H)
            gst(spec, e, v[s]);
        else if (e == H)
            gst(static_cast<cplx<T>*>(m.spec_nyq), q, v[s]);
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
template <class P, typename T, bool INV, bool STRIDED>
__device__ __forceinline__ void transform_tile(cplx<T>* data, const Strides& sd, int64_t tile,
                                               cplx<T>* lds, const cplx<T>* tw) {
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

// P2 / P4 (psi) and P6 / P8 (half spectrum + Nyquist plane).
template <int NY, typename T, bool INV, bool SPEC>
__global__ __launch_bounds__((wg_size<typename PlanFor<NY>::type, T>())) void k_y_fft(
    const MemberDev* __restrict__ mems, int first) {
    using FP = typename PlanFor<NY>::type;
    constexpr int PP = pencils_per_wg<FP, T>();
    __shared__ cplx<T> lds[lds_entries<FP, T, !SPEC>()];
    __shared__ cplx<T> tw[tw_entries<T>(NY)];
    const MemberDev& m = mems[first + blockIdx.y];
    load_twiddles<NY, wg_size<FP, T>()>(tw, m.tw_y);
    __syncthreads();
    const int64_t nx = m.nx, ny = m.ny, nz = m.nz;
    if constexpr (!SPEC) {
        const Strides sd{nx * nz, nz, ny * nz, nz};
        transform_tile<FP, T, INV, true>(static_cast<cplx<T>*>(m.psi), sd, blockIdx.x, lds, tw);
    } else {
        const int64_t h = nz / 2;
        const int64_t main_tiles = (nx * h + PP - 1) / PP;
        if (int64_t(blockIdx.x) < main_tiles) {
            const Strides sd{nx * h, h, ny * h, h};
            transform_tile<FP, T, INV, true>(static_cast<cplx<T>*>(m.spec), sd, blockIdx.x, lds,
                                             tw);
        } else {
            // kz = nz/2 plane [nx][ny]: y-pencils are contiguous
            const Strides sd{nx, 1, ny, 1};
            transform_tile<FP, T, INV, false>(static_cast<cplx<T>*>(m.spec_nyq), sd,
                                              blockIdx.x - main_tiles, lds, tw);
        }
    }
}

// P3: x forward, kinetic phase, x inverse, with the factor tables P1 wrote
// for this step: complex64 multiplies by each hi + lo pair with one rounding
// (cmul_split), first by e_x, then by e_yz; complex128 by the FP64 product.
template <int NX, typename T>
__global__ __launch_bounds__((wg_size<typename PlanFor<NX>::type, T>())) void k_x_kinetic(
    const MemberDev* __restrict__ mems, int first) {
    using FP = typename PlanFor<NX>::type;
    using IP = Reversed<FP>;
    using LN = Lanes<FP, T, true>;
    constexpr int WG = wg_size<FP, T>();
    constexpr bool kSplit = std::is_same<T, float>::value;
    __shared__ cplx<T> lds[lds_entries<FP, T, true>()];
    __shared__ cplx<T> tw[tw_entries<T>(NX)];
    // complex64: hi in [0, NX), lo in [NX, 2 NX); complex128: the factor
    __shared__ cplx<T> ex[kSplit ? 2 * NX : NX];
    const MemberDev& m = mems[first + blockIdx.y];
    load_twiddles<NX, WG>(tw, m.tw_x);
    const cplx<T>* kin = static_cast<const cplx<T>*>(m.kin);
    constexpr int KE = kSplit ? 2 * NX : NX;   // complex entries of e_x
    constexpr int KI = (KE + WG - 1) / WG;
    cplx<T> kr[KI];
#pragma unroll
    for (int k = 0; k < KI; ++k) {
        const int i = int(threadIdx.x) + k * WG;
        kr[k] = (KE % WG == 0 || i < KE) ? gld(kin, i) : cplx<T>{T(0), T(0)};
    }
    const LN ln;
    const int64_t ny = m.ny, nz = m.nz;
    const int64_t plane = ny * nz;
    const int64_t q = int64_t(blockIdx.x) * LN::PP + ln.p;
    const bool ok = q < plane;
    // this pencil's e_yz
    const int64_t qe = NX + (ok ? q : 0);
    const cplx<T> yh = gld(kin, kSplit ? 2 * qe : qe);
    const cplx<T> yl = kSplit ? gld(kin, 2 * qe + 1) : cplx<T>{T(0), T(0)};
    cplx<T>* psi = static_cast<cplx<T>*>(m.psi);
    cplx<T> v[FP::E];
    load_slots<FP, FP::first()>(v, psi, q, plane, ok, ln);
#pragma unroll
    for (int k = 0; k < KI; ++k) {
        const int i = int(threadIdx.x) + k * WG;
        if (KE % WG == 0 || i < KE) {
            // complex64 entries alternate hi, lo
            if constexpr (kSplit)
                ex[(i & 1) * NX + (i >> 1)] = kr[k];
            else
                ex[i] = kr[k];
        }
    }
    __syncthreads();
    pencil_fft<FP, false, T>(v, lds, tw, ln.t, ln);
    if constexpr (kSplit) {
#pragma unroll
        for (int s = 0; s < FP::E; ++s) {
            const int e = slot_elem<FP, FP::last()>(ln.t, s);
            v[s] = cmul_split(cmul_split(v[s], ex[e], ex[NX + e]), yh, yl);
        }
    } else {
#pragma unroll
        for (int s = 0; s < FP::E; ++s)
            v[s] = cmul(v[s], cmul(ex[slot_elem<FP, FP::last()>(ln.t, s)], yh));
    }
    __syncthreads();
    pencil_fft<IP, true, T>(v, lds, tw, ln.t, ln);
    store_slots<IP, IP::last()>(v, psi, q, plane, ok, ln);
}

// 1 / x for normal x: hardware reciprocal refined by one Newton step in single
// precision (within about one unit in the last place); FP64 division otherwise.
__device__ __forceinline__ float recip(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(fmaf(-x, r, 1.0f), r, r);
}
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// P7: x forward, Green's function, x inverse, on the half spectrum and the
// Nyquist plane.  |k|^2 is summed in FP64 from a per-work-group table of k_x^2;
// the quotient -4 pi G / (|k|^2 N) is taken in the grid precision (its
// rounding perturbs Phi by one unit in the last place, recomputed every step).
template <int NX, typename T>
__global__ __launch_bounds__((wg_size<typename PlanFor<NX>::type, T>())) void k_x_green(
    const MemberDev* __restrict__ mems, int first) {
    using FP = typename PlanFor<NX>::type;
    using IP = Reversed<FP>;
    using LN = Lanes<FP, T, true>;
    __shared__ cplx<T> lds[lds_entries<FP, T, true>()];
    __shared__ cplx<T> tw[tw_entries<T>(NX)];
    __shared__ double kx2[NX];
    const MemberDev& m = mems[first + blockIdx.y];
    load_twiddles<NX, wg_size<FP, T>()>(tw, m.tw_x);
    const double cx = kTwoPi / m.lx, cy = kTwoPi / m.ly, cz = kTwoPi / m.lz;
    for (int i = int(threadIdx.x); i < NX; i += int(blockDim.x)) {
        const double kx = cx * signed_mode(i, NX);
        kx2[i] = kx * kx;
    }
    __syncthreads();
    const LN ln;
    const int64_t ny = m.ny, h = m.nz / 2;
    const int64_t main_tiles = (ny * h + LN::PP - 1) / LN::PP;
    const bool nyq = int64_t(blockIdx.x) >= main_tiles;
    const int64_t tile = nyq ? blockIdx.x - main_tiles : blockIdx.x;
    const int64_t plane = nyq ? ny : ny * h;
    const int64_t q = tile * LN::PP + ln.p;
    const bool ok = q < plane;
    const int64_t iy = nyq ? q : q / h;
    const int64_t iz = nyq ? h : q % h;
    const double ky = cy * signed_mode(int(iy), int(ny));
    const double kz = cz * double(iz);
    const double kyz2 = ky * ky + kz * kz;
    const T gscale = T(-m.four_pi_G / (double(m.nx) * double(ny) * double(m.nz)));
    cplx<T>* data = static_cast<cplx<T>*>(nyq ? m.spec_nyq : m.spec);
    cplx<T> v[FP::E];
    load_slots<FP, FP::first()>(v, data, q, plane, ok, ln);
    pencil_fft<FP, false, T>(v, lds, tw, ln.t, ln);
#pragma unroll
    for (int s = 0; s < FP::E; ++s) {
        const T k2 = T(kx2[slot_elem<FP, FP::last()>(ln.t, s)] + kyz2);
        v[s] = cscale(v[s], k2 > T(0) ? gscale * recip(k2) : T(0));
    }
    __syncthreads();
    pencil_fft<IP, true, T>(v, lds, tw, ln.t, ln);
    store_slots<IP, IP::last()>(v, data, q, plane, ok, ln);
}

// Plain axis transform of psi or scratch (diagnostics, tests of the FFT).
template <int N, typename T, bool INV, int AXIS>
__global__ __launch_bounds__((wg_size<typename PlanFor<N>::type, T>())) void k_axis_fft(
    const MemberDev* __restrict__ mems, int first, int which) {
    using FP = typename PlanFor<N>::type;
    __shared__ cplx<T> lds[lds_entries<FP, T, false>()];
    __shared__ cplx<T> tw[tw_entries<T>(N)];
    const MemberDev& m = mems[first + blockIdx.y];
    load_twiddles<N, wg_size<FP, T>()>(tw, AXIS == 0 ? m.tw_x : (AXIS == 1 ? m.tw_y : m.tw_z));
    __syncthreads();
    cplx<T>* data = static_cast<cplx<T>*>(which ? m.scratch : m.psi);
    const int64_t nx = m.nx, ny = m.ny, nz = m.nz;
    if constexpr (AXIS == 2) {
        const Strides sd{nx * ny, 1, nz, 1};
        transform_tile<FP, T, INV, false>(data, sd, blockIdx.x, lds, tw);
    } else if constexpr (AXIS == 1) {
        const Strides sd{nx * nz, nz, ny * nz, nz};
        transform_tile<FP, T, INV, true>(data, sd, blockIdx.x, lds, tw);
    } else {
        const Strides sd{ny * nz, ny * nz, 0, ny * nz};
        transform_tile<FP, T, INV, true>(data, sd, blockIdx.x, lds, tw);
    }
}

// Spectral kinetic energy: x forward FFT of scratch (already z and y
// transformed) and FP64 partial sums of |k|^2 |psi_k|^2 per work-group.
template <int NX, typename T>
__global__ __launch_bounds__((wg_size<typename PlanFor<NX>::type, T>())) void k_x_kinetic_energy(
    const MemberDev* __restrict__ mems, int first) {
    using FP = typename PlanFor<NX>::type;
    using LN = Lanes<FP, T, true>;
    constexpr int WG = wg_size<FP, T>();
    __shared__ cplx<T> lds[lds_entries<FP, T, true>()];
    __shared__ cplx<T> tw[tw_entries<T>(NX)];
    __shared__ double red[WG];
    const MemberDev& m = mems[first + blockIdx.y];
    load_twiddles<NX, wg_size<FP, T>()>(tw, m.tw_x);
    __syncthreads();
    const LN ln;
    const int64_t ny = m.ny, nz = m.nz, plane = ny * nz;
    const int64_t q = int64_t(blockIdx.x) * LN::PP + ln.p;
    const bool ok = q < plane;
    cplx<T> v[FP::E];
    load_slots<FP, FP::first()>(v, static_cast<cplx<T>*>(m.scratch), q, plane, ok, ln);
    pencil_fft<FP, false, T>(v, lds, tw, ln.t, ln);
    const double cx = kTwoPi / m.lx, cy = kTwoPi / m.ly, cz = kTwoPi / m.lz;
    const double ky = cy * signed_mode(int(q / nz), int(ny));
    const double kz = cz * signed_mode(int(q % nz), int(nz));
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < FP::E; ++s) {
        const double kx = cx * signed_mode(slot_elem<FP, FP::last()>(ln.t, s), NX);
        const double a2 = double(v[s].re) * double(v[s].re) + double(v[s].im) * double(v[s].im);
        acc += (kx * kx + ky * ky + kz * kz) * a2;
    }
    red[threadIdx.x] = ok ? acc : 0.0;
    __syncthreads();
    for (int w = WG / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) gstr(m.partials, int64_t(blockIdx.x) * kRedFields + 1, red[0]);
}

// ---------------------------------------------------------------------------
// host launchers: dispatch on the axis length
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

template <int N, typename T>
static int64_t tiles(int64_t pencils) {
    using FP = typename PlanFor<N>::type;
    constexpr int PP = pencils_per_wg<FP, T>();
    return (pencils + PP - 1) / PP;
}
template <int N, typename T>
static dim3 block() {
    return dim3(wg_size<typename PlanFor<N>::type, T>());
}

template <int NZ>
struct ZPotKick {
    template <typename T>
    static hipError_t go(const Launch& L, int nx, int ny, ZOp op, KickMode k) {
        dim3 grid(unsigned(tiles<NZ, T>(int64_t(nx) * ny)), unsigned(L.count));
        if (op == kZPhiOnly)
            k_z_potential_kick<NZ, T, kZPhiOnly, kHalfKick>
                <<<grid, block<NZ, T>(), 0, L.stream>>>(L.members, L.first);
        else if (op == kZKickOnly && k == kHalfKick)
            k_z_potential_kick<NZ, T, kZKickOnly, kHalfKick>
                <<<grid, block<NZ, T>(), 0, L.stream>>>(L.members, L.first);
        else if (op == kZKickOnly)
            k_z_potential_kick<NZ, T, kZKickOnly, kFullKick>
                <<<grid, block<NZ, T>(), 0, L.stream>>>(L.members, L.first);
        else if (k == kHalfKick)
            k_z_potential_kick<NZ, T, kZKickFft, kHalfKick>
                <<<grid, block<NZ, T>(), 0, L.stream>>>(L.members, L.first);
        else
            k_z_potential_kick<NZ, T, kZKickFft, kFullKick>
                <<<grid, block<NZ, T>(), 0, L.stream>>>(L.members, L.first);
        return hipGetLastError();
    }
    static hipError_t run(const Launch& L, int prec, int nx, int ny, ZOp op, KickMode k) {
        return prec ? go<double>(L, nx, ny, op, k) : go<float>(L, nx, ny, op, k);
    }
};

template <int NZ>
struct ZDens {
    template <typename T>
    static hipError_t go(const Launch& L, int nx, int ny, DensOp op) {
        dim3 grid(unsigned(tiles<NZ, T>(int64_t(nx) * ny)), unsigned(L.count));
        if (op == kDensInvFft)
            k_z_density<NZ, T, kDensInvFft><<<grid, block<NZ, T>(), 0, L.stream>>>(L.members, L.first);
        else
            k_z_density<NZ, T, kDensDirect><<<grid, block<NZ, T>(), 0, L.stream>>>(L.members, L.first);
        return hipGetLastError();
    }
    static hipError_t run(const Launch& L, int prec, int nx, int ny, DensOp op) {
        return prec ? go<double>(L, nx, ny, op) : go<float>(L, nx, ny, op);
    }
};

template <int NY>
struct YFft {
    template <typename T>
    static hipError_t go(const Launch& L, int nx, int nz, bool inv, bool spec) {
        int64_t t;
        if (spec)
            t = tiles<NY, T>(int64_t(nx) * (nz / 2)) + tiles<NY, T>(nx);
        else
            t = tiles<NY, T>(int64_t(nx) * nz);
        dim3 grid(unsigned(t), unsigned(L.count));
        auto b = block<NY, T>();
        if (spec) {
            if (inv)
                k_y_fft<NY, T, true, true><<<grid, b, 0, L.stream>>>(L.members, L.first);
            else
                k_y_fft<NY, T, false, true><<<grid, b, 0, L.stream>>>(L.members, L.first);
        } else {
            if (inv)
                k_y_fft<NY, T, true, false><<<grid, b, 0, L.stream>>>(L.members, L.first);
            else
                k_y_fft<NY, T, false, false><<<grid, b, 0, L.stream>>>(L.members, L.first);
        }
        return hipGetLastError();
    }
    static hipError_t run(const Launch& L, int prec, int nx, int nz, bool inv, bool spec) {
        return prec ? go<double>(L, nx, nz, inv, spec) : go<float>(L, nx, nz, inv, spec);
    }
};

template <int NX>
struct XKin {
    template <typename T>
    static hipError_t go(const Launch& L, int ny, int nz) {
        dim3 grid(unsigned(tiles<NX, T>(int64_t(ny) * nz)), unsigned(L.count));
        k_x_kinetic<NX, T><<<grid, block<NX, T>(), 0, L.stream>>>(L.members, L.first);
        return hipGetLastError();
    }
    static hipError_t run(const Launch& L, int prec, int ny, int nz) {
        return prec ? go<double>(L, ny, nz) : go<float>(L, ny, nz);
    }
};

template <int NX>
struct XGreen {
    template <typename T>
    static hipError_t go(const Launch& L, int ny, int nz) {
        const int64_t t = tiles<NX, T>(int64_t(ny) * (nz / 2)) + tiles<NX, T>(ny);
        dim3 grid(unsigned(t), unsigned(L.count));
        k_x_green<NX, T><<<grid, block<NX, T>(), 0, L.stream>>>(L.members, L.first);
        return hipGetLastError();
    }
    static hipError_t run(const Launch& L, int prec, int ny, int nz) {
        return prec ? go<double>(L, ny, nz) : go<float>(L, ny, nz);
    }
};

template <int N>
struct AxisFft {
    template <typename T, bool INV>
    static hipError_t go2(const Launch& L, int64_t pencils, int axis, int which) {
        dim3 grid(unsigned(tiles<N, T>(pencils)), unsigned(L.count));
        auto b = block<N, T>();
        if (axis == 0)
            k_axis_fft<N, T, INV, 0><<<grid, b, 0, L.stream>>>(L.members, L.first, which);
        else if (axis == 1)
            k_axis_fft<N, T, INV, 1><<<grid, b, 0, L.stream>>>(L.members, L.first, which);
        else
            k_axis_fft<N, T, INV, 2><<<grid, b, 0, L.stream>>>(L.members, L.first, which);
        return hipGetLastError();
    }
    static hipError_t run(const Launch& L, int prec, int64_t pencils, int axis, bool inv,
                          int which) {
        if (prec)
            return inv ? go2<double, true>(L, pencils, axis, which)
                       : go2<double, false>(L, pencils, axis, which);
        return inv ? go2<float, true>(L, pencils, axis, which)
                   : go2<float, false>(L, pencils, axis, which);
    }
};

template <int NX>
struct XKinE {
    template <typename T>
    static hipError_t go(const Launch& L, int ny, int nz) {
        dim3 grid(unsigned(tiles<NX, T>(int64_t(ny) * nz)), 1u);
        k_x_kinetic_energy<NX, T><<<grid, block<NX, T>(), 0, L.stream>>>(L.members, L.first);
        return hipGetLastError();
    }
    static hipError_t run(const Launch& L, int prec, int ny, int nz) {
        return prec ? go<double>(L, ny, nz) : go<float>(L, ny, nz);
    }
};

hipError_t launch_z_potential_kick(const Launch& L, int prec, int nx, int ny, int nz, ZOp op,
                                   KickMode kick) {
    return dispatch_n<ZPotKick>(nz, L, prec, nx, ny, op, kick);
}
hipError_t launch_z_density(const Launch& L, int prec, int nx, int ny, int nz, DensOp op) {
    return dispatch_n<ZDens>(nz, L, prec, nx, ny, op);
}
hipError_t launch_y_fft_psi(const Launch& L, int prec, int nx, int ny, int nz, bool inverse) {
    return dispatch_n<YFft>(ny, L, prec, nx, nz, inverse, false);
}
hipError_t launch_y_fft_spec(const Launch& L, int prec, int nx, int ny, int nz, bool inverse) {
    return dispatch_n<YFft>(ny, L, prec, nx, nz, inverse, true);
}
hipError_t launch_x_kinetic(const Launch& L, int prec, int nx, int ny, int nz) {
    return dispatch_n<XKin>(nx, L, prec, ny, nz);
}
hipError_t launch_x_green(const Launch& L, int prec, int nx, int ny, int nz) {
    return dispatch_n<XGreen>(nx, L, prec, ny, nz);
}
hipError_t launch_axis_fft(const Launch& L, int prec, int nx, int ny, int nz, int axis,
                           bool inverse, int which) {
    const int n = axis == 0 ? nx : (axis == 1 ? ny : nz);
    const int64_t pencils = axis == 0 ? int64_t(ny) * nz
                                      : (axis == 1 ? int64_t(nx) * nz : int64_t(nx) * ny);
    return dispatch_n<AxisFft>(n, L, prec, pencils, axis, inverse, which);
}
hipError_t launch_x_kinetic_energy(const Launch& L, int prec, int nx, int ny, int nz) {
    return dispatch_n<XKinE>(nx, L, prec, ny, nz);
}

int64_t axis_tiles(int n, int64_t pencils, int prec) {
#define WDM_TILES_CASE(N) \
    case N: return prec ? tiles<N, double>(pencils) : tiles<N, float>(pencils);
    switch (n) {
        WDM_TILES_CASE(16)
        WDM_TILES_CASE(32)
        WDM_TILES_CASE(64)
        WDM_TILES_CASE(96)
        WDM_TILES_CASE(128)
        WDM_TILES_CASE(192)
        WDM_TILES_CASE(256)
        WDM_TILES_CASE(384)
        WDM_TILES_CASE(512)
        default: return 0;
    }
#undef WDM_TILES_CASE
}

}  // namespace wdm
