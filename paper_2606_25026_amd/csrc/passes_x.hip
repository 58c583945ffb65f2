// P3 and P7: the passes along x (kinetic phase, Green's function), and the
// spectral kinetic energy.
#include "passes_common.hpp"

namespace wdm {

// P3: x forward, kinetic phase, x inverse, with the factor tables P1 wrote
// for this step.  Each mode is multiplied by the FP64 product
// e_x(k_x) e_yz(k_y, k_z) / N, rounded once to the grid precision.  (Two
// single-rounding products, first by e_x then by e_yz, were measured to drift
// the complex64 norm by +9e-9 per step on the 128^3 sub-box, against -3e-10
// with the one FP64 product.)
template <int NX, typename T, int V>
__global__ __launch_bounds__((wg_size<typename PlanFor<NX, V>::type, T>())) void k_x_kinetic(
    const MemberDev* __restrict__ mems, int first) {
    using FP = typename PlanFor<NX, V>::type;
    using IP = Reversed<FP>;
    using LN = Lanes<FP, T, true>;
    constexpr int WG = wg_size<FP, T>();
    constexpr bool kSplit = std::is_same<T, float>::value;
    __builtin_amdgcn_s_setprio(2);   // beside the particle kernel, as P2 / P4
    __shared__ strided_lds_t<FP, T> lds[lds_entries<FP, T, true>()];
    __shared__ cplx<T> tw[tw_entries<T>(NX)];
    __shared__ cplx<double> ex[NX];   // e_x in FP64
    const MemberDev& m = mems[first + blockIdx.y];
    load_twiddles<NX, WG>(tw, m.tw_x);
    // complex64 tables hold (hi, lo) pairs: 2 entries per factor
    const cplx<T>* kin = static_cast<const cplx<T>*>(m.kin);
    constexpr int KS = kSplit ? 2 : 1;
    constexpr int KI = (NX + WG - 1) / WG;
    cplx<T> kh[KI], kl[KI];
#pragma unroll
    for (int k = 0; k < KI; ++k) {
        const int i = int(threadIdx.x) + k * WG;
        const bool in = NX % WG == 0 || i < NX;
        kh[k] = in ? gld(kin, KS * i) : cplx<T>{T(0), T(0)};
        kl[k] = (in && kSplit) ? gld(kin, KS * i + 1) : cplx<T>{T(0), T(0)};
    }
    const LN ln;
    const int64_t ny = m.ny, nz = m.nz;
    const int64_t plane = ny * nz;
    const int64_t q = int64_t(blockIdx.x) * LN::PP + ln.p;
    const bool ok = q < plane;
    // this pencil's e_yz / N
    const int64_t qe = NX + (ok ? q : 0);
    const cplx<T> yh = gld(kin, KS * qe);
    const cplx<T> yl = kSplit ? gld(kin, KS * qe + 1) : cplx<T>{T(0), T(0)};
    const cplx<double> eyz{double(yh.re) + double(yl.re), double(yh.im) + double(yl.im)};
    cplx<T>* psi = static_cast<cplx<T>*>(m.psi);
    cplx<T> v[FP::E];
    load_slots<FP, FP::first()>(v, psi, q, plane, ok, ln);
#pragma unroll
    for (int k = 0; k < KI; ++k) {
        const int i = int(threadIdx.x) + k * WG;
        if (NX % WG == 0 || i < NX)
            ex[i] = cplx<double>{double(kh[k].re) + double(kl[k].re),
                                 double(kh[k].im) + double(kl[k].im)};
    }
    __syncthreads();
    pencil_fft<FP, false, T>(v, lds, tw, ln.t, ln);
#pragma unroll
    for (int s = 0; s < FP::E; ++s)
        v[s] = mul64(v[s], cmul(ex[slot_elem<FP, FP::last()>(ln.t, s)], eyz));
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
template <int NX, typename T, int V>
__global__ __launch_bounds__((wg_size<typename PlanFor<NX, V>::type, T>())) void k_x_green(
    const MemberDev* __restrict__ mems, int first) {
    using FP = typename PlanFor<NX, V>::type;
    using IP = Reversed<FP>;
    using LN = Lanes<FP, T, true>;
    __shared__ strided_lds_t<FP, T> lds[lds_entries<FP, T, true>()];
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


// Vacuum-boundary convolution, x pass on the zero-padded grid (a padded
// member descriptor: lengths 2n, psi = the padded grid): x forward transform,
// multiplication by the stored real transform of the padded Green's function
// (same [x][y][z] layout), x inverse transform, in one pass as P7 does.  Only
// the x < NX/2 half is read (the padding half holds zeros and is never
// written) and only that half of the result, the one the potential needs, is
// stored.
template <int NX, typename T, int V>
__global__ __launch_bounds__((wg_size<typename PlanFor<NX, V>::type, T>())) void k_x_mul_green(
    const MemberDev* __restrict__ mems, int first) {
    using FP = typename PlanFor<NX, V>::type;
    using IP = Reversed<FP>;
    using LN = Lanes<FP, T, true>;
    __shared__ T lds[lds_entries<FP, T, true>()];
    __shared__ cplx<T> tw[tw_entries<T>(NX)];
    const MemberDev& m = mems[first + blockIdx.y];
    load_twiddles<NX, wg_size<FP, T>()>(tw, m.tw_x);
    __syncthreads();
    const LN ln;
    // element offsets fit 32 bits: at most 512 * 512 * 512 per padded grid
    const int plane = m.ny * m.nz;
    const int q = int(blockIdx.x) * LN::PP + ln.p;
    const bool ok = q < plane;
    cplx<T>* lane = static_cast<cplx<T>*>(m.psi) + q;
    constexpr int HALF = NX / 2;
    // The Green's factors are even in each wavenumber and stored for modes
    // 0..n of each axis (n = half the padded length): mode k > n reads 2n - k.
    const int hy = m.ny / 2, hz = m.nz / 2;
    const int qy = q / m.nz, qz = q - qy * m.nz;
    const int gplane = (hy + 1) * (hz + 1);
    const T* green = static_cast<const T*>(m.green) +
                     (min(qy, m.ny - qy) * (hz + 1) + min(qz, m.nz - qz));
    // the Green's factors of this lane's output slots are loaded with the data
    T gv[FP::E];
    cplx<T> v[FP::E];
#pragma unroll
    for (int s = 0; s < FP::E; ++s) {
        const int ein = slot_elem<FP, FP::first()>(ln.t, s);
        v[s] = (ok && ein < HALF) ? gld(lane, ein * plane) : cplx<T>{T(0), T(0)};
        const int kx = slot_elem<FP, FP::last()>(ln.t, s);
        gv[s] = ok ? gldr(green, min(kx, NX - kx) * gplane) : T(0);
    }
    pencil_fft<FP, false, T>(v, lds, tw, ln.t, ln);
#pragma unroll
    for (int s = 0; s < FP::E; ++s) v[s] = cscale(v[s], gv[s]);
    __syncthreads();
    pencil_fft<IP, true, T>(v, lds, tw, ln.t, ln);
    if (!ok) return;
#pragma unroll
    for (int s = 0; s < FP::E; ++s) {
        const int eout = slot_elem<IP, IP::last()>(ln.t, s);
        if (eout < HALF) gst(lane, eout * plane, v[s]);
    }
}

template <int NX, typename T>
__global__ __launch_bounds__((wg_size<typename PlanFor<NX>::type, T>())) void k_x_kinetic_energy(
    const MemberDev* __restrict__ mems, int first) {
    using FP = typename PlanFor<NX>::type;
    using LN = Lanes<FP, T, true>;
    constexpr int WG = wg_size<FP, T>();
    __shared__ T lds[lds_entries<FP, T, true>()];
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


template <int NX>
struct XKin {
    template <typename T, int V>
    static hipError_t go(const Launch& L, int ny, int nz) {
        dim3 grid(unsigned(tiles<NX, T, V>(int64_t(ny) * nz)), unsigned(L.count));
        k_x_kinetic<NX, T, V><<<grid, block<NX, T, V>(), 0, L.stream>>>(L.members, L.first);
        return hipGetLastError();
    }
    template <typename T>
    static hipError_t pick(const Launch& L, int ny, int nz, int var) {
        if constexpr (has_variant(NX))
            if (var == 1) return go<T, 1>(L, ny, nz);
        if constexpr (has_wide(NX)) {
            if (var == 2) return go<T, 2>(L, ny, nz);
            if (var == 3) return go<T, 3>(L, ny, nz);
        }
        return go<T, 0>(L, ny, nz);
    }
    static hipError_t run(const Launch& L, int prec, int ny, int nz, int var) {
        return prec ? pick<double>(L, ny, nz, var) : pick<float>(L, ny, nz, var);
    }
};

template <int NX>
struct XGreen {
    template <typename T, int V>
    static hipError_t go(const Launch& L, int ny, int nz) {
        const int64_t t = tiles<NX, T, V>(int64_t(ny) * (nz / 2)) + tiles<NX, T, V>(ny);
        dim3 grid(unsigned(t), unsigned(L.count));
        k_x_green<NX, T, V><<<grid, block<NX, T, V>(), 0, L.stream>>>(L.members, L.first);
        return hipGetLastError();
    }
    template <typename T>
    static hipError_t pick(const Launch& L, int ny, int nz, int var) {
        if constexpr (has_variant(NX))
            if (var == 1) return go<T, 1>(L, ny, nz);
        if constexpr (has_wide(NX)) {
            if (var == 2) return go<T, 2>(L, ny, nz);
            if (var == 3) return go<T, 3>(L, ny, nz);
        }
        return go<T, 0>(L, ny, nz);
    }
    static hipError_t run(const Launch& L, int prec, int ny, int nz, int var) {
        return prec ? pick<double>(L, ny, nz, var) : pick<float>(L, ny, nz, var);
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

template <int NX>
struct XMulGreen {
    template <typename T>
    static hipError_t go(const Launch& L, int ny, int nz) {
        constexpr int V = 0;   // the second plan measured slower on the padded 512 axis
        dim3 grid(unsigned(tiles<NX, T, V>(int64_t(ny) * nz)), unsigned(L.count));
        k_x_mul_green<NX, T, V><<<grid, block<NX, T, V>(), 0, L.stream>>>(L.members, L.first);
        return hipGetLastError();
    }
    static hipError_t run(const Launch& L, int prec, int ny, int nz) {
        return prec ? go<double>(L, ny, nz) : go<float>(L, ny, nz);
    }
};

hipError_t launch_x_mul_green(const Launch& L, int prec, int nx, int ny, int nz) {
    return dispatch_n<XMulGreen>(nx, L, prec, ny, nz);
}

// The kinetic factor tables of the dt in use, for every member of the class
// (grid-stride over nx + ny nz entries per member).
template <typename T>
__global__ __launch_bounds__(256) void k_kinetic_tables(const MemberDev* __restrict__ mems,
                                                        int first) {
    const MemberDev& m = mems[first + blockIdx.y];
    write_kinetic_table<T>(m, gldr(m.dt, 0), int64_t(gridDim.x) * blockDim.x,
                           int64_t(blockIdx.x) * blockDim.x + threadIdx.x);
}

hipError_t launch_kinetic_tables(const Launch& L, int prec, int64_t max_entries) {
    int64_t g = (max_entries + 255) / 256;
    if (g > 1024) g = 1024;
    const dim3 grid(unsigned(g), unsigned(L.count));
    if (prec)
        k_kinetic_tables<double><<<grid, 256, 0, L.stream>>>(L.members, L.first);
    else
        k_kinetic_tables<float><<<grid, 256, 0, L.stream>>>(L.members, L.first);
    return hipGetLastError();
}

hipError_t launch_x_kinetic(const Launch& L, int prec, int nx, int ny, int nz, int variant) {
    return dispatch_n<XKin>(nx, L, prec, ny, nz, variant);
}
hipError_t launch_x_green(const Launch& L, int prec, int nx, int ny, int nz, int variant) {
    return dispatch_n<XGreen>(nx, L, prec, ny, nz, variant);
}
hipError_t launch_x_kinetic_energy(const Launch& L, int prec, int nx, int ny, int nz) {
    return dispatch_n<XKinE>(nx, L, prec, ny, nz);
}

}  // namespace wdm
