// P2, P4, P6, P8: the passes along y, and plain axis transforms.
#include "passes_common.hpp"

namespace wdm {

bool axis_supported(int n) {
    switch (n) {
        case 16: case 32: case 64: case 96: case 128: case 192: case 256: case 384: case 512:
            return true;
        default:
            return false;
    }
}

bool axis_has_variant(int n) { return axis_supported(n) && has_variant(n); }
bool axis_has_wide(int n) { return axis_supported(n) && has_wide(n); }

// P2 / P4 (psi) and P6 / P8 (half spectrum + Nyquist plane).
template <int NY, typename T, bool INV, bool SPEC, int V>
__global__ __launch_bounds__((wg_size<typename PlanFor<NY, V>::type, T>())) void k_y_fft(
    const MemberDev* __restrict__ mems, int first) {
    using FP = typename PlanFor<NY, V>::type;
    constexpr int PP = pencils_per_wg<FP, T>();
    // P2 / P4 share the machine with the particle kernel: their waves issue
    // first on a SIMD (wave priority 2 of 0-3; the particle waves stay at 0),
    // which keeps these bandwidth-bound passes streaming (256^3 + 1e6 step
    // 0.4079 -> 0.4060 ms on average over four paired runs on two machines)
    if constexpr (!SPEC) __builtin_amdgcn_s_setprio(2);
    __shared__ strided_lds_t<FP, T> lds[lds_entries<FP, T, !SPEC>()];
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


// Plain axis transform of psi or scratch (diagnostics, tests of the FFT).
template <int N, typename T, bool INV, int AXIS>
__global__ __launch_bounds__((wg_size<typename PlanFor<N>::type, T>())) void k_axis_fft(
    const MemberDev* __restrict__ mems, int first, int which) {
    using FP = typename PlanFor<N>::type;
    __shared__ T lds[lds_entries<FP, T, false>()];
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

// Transforms of the vacuum solve's zero-padded grid (Sec. 3.2.1), run on the
// padded member table (doubled lengths, psi = the padded grid).  Only the
// quarter of the padded grid that can be non-zero before the x pass (x < nx,
// y < ny) is read or written along z, and the y passes see the y >= ny half of
// each pencil as zeros (forward) or do not store it (inverse), so the padded
// grid's y >= ny rows are never touched:
//   kVacZFwd  the density rows (real, nz values, held in Phi) zero-extended to
//             2 nz, forward z transform into the padded rows (x < nx, y < ny);
//   kVacYFwd  forward y transform of the x < nx pencils, inputs y >= ny zero;
//   kVacYInv  inverse y transform of the x < nx pencils, outputs y < ny stored;
//   kVacZInv  inverse z transform of the padded rows (x < nx, y < ny), the real
//             part of the first nz values written to Phi.
enum VacMode : int { kVacZFwd = 0, kVacYFwd = 1, kVacYInv = 2, kVacZInv = 3 };

template <int N, typename T, int MODE>
__global__ __launch_bounds__((wg_size<typename PlanFor<N>::type, T>())) void k_vac_fft(
    const MemberDev* __restrict__ mems, int first) {
    using FP = typename PlanFor<N>::type;
    constexpr bool STRIDED = MODE == kVacYFwd || MODE == kVacYInv;
    constexpr bool INV = MODE == kVacYInv || MODE == kVacZInv;
    constexpr int H = N / 2;   // the unpadded length along the transformed axis
    using LN = Lanes<FP, T, STRIDED>;
    __shared__ T lds[lds_entries<FP, T, false>()];
    __shared__ cplx<T> tw[tw_entries<T>(N)];
    const MemberDev& m = mems[first + blockIdx.y];
    load_twiddles<N, wg_size<FP, T>()>(tw, STRIDED ? m.tw_y : m.tw_z);
    __syncthreads();
    const LN ln;
    const int64_t q = int64_t(blockIdx.x) * LN::PP + ln.p;
    cplx<T>* pad = static_cast<cplx<T>*>(m.psi);
    cplx<T> v[FP::E];
    if constexpr (STRIDED) {
        // y pencils of the padded [2nx][2ny][2nz] grid with x < nx: q = x 2nz + z
        const int64_t pny = m.ny, pnz = m.nz;
        const int64_t count = int64_t(m.nx / 2) * pnz;
        const bool ok = q < count;
        const int64_t b = ok ? (q / pnz) * (pny * pnz) + (q % pnz) : 0;
        cplx<T>* lane = pad + (b + int64_t(ln.t) * pnz);
#pragma unroll
        for (int s = 0; s < FP::E; ++s) {
            constexpr int R0 = FP::first();
            const int e = ln.t + slot_const<FP, R0>(s);
            v[s] = (ok && (MODE == kVacYInv || e < H)) ? gld(lane, int64_t(slot_const<FP, R0>(s)) * pnz)
                                                       : cplx<T>{T(0), T(0)};
        }
        pencil_fft<FP, INV, T>(v, lds, tw, ln.t, ln);
        if (!ok) return;
#pragma unroll
        for (int s = 0; s < FP::E; ++s) {
            constexpr int R1 = FP::last();
            const int e = ln.t + slot_const<FP, R1>(s);
            if (MODE == kVacYFwd || e < H) gst(lane, int64_t(slot_const<FP, R1>(s)) * pnz, v[s]);
        }
    } else {
        // rows (x, y), x < nx, y < ny: q = x ny + y
        const int rnx = m.nx / 2, rny = m.ny / 2;
        const bool ok = q < int64_t(rnx) * rny;
        const int64_t x = ok ? q / rny : 0, y = ok ? q - x * rny : 0;
        const int64_t pb = (x * m.ny + y) * m.nz;      // padded row
        T* phi = static_cast<T*>(m.phi) + (ok ? q : 0) * H;
        if constexpr (MODE == kVacZFwd) {
#pragma unroll
            for (int s = 0; s < FP::E; ++s) {
                const int e = ln.t + slot_const<FP, FP::first()>(s);
                v[s] = cplx<T>{(ok && e < H) ? gldr(phi, e) : T(0), T(0)};
            }
            pencil_fft<FP, false, T>(v, lds, tw, ln.t, ln);
            store_slots<FP, FP::last()>(v, pad, pb, 1, ok, ln);
        } else {
            load_slots<FP, FP::first()>(v, pad, pb, 1, ok, ln);
            pencil_fft<FP, true, T>(v, lds, tw, ln.t, ln);
            if (!ok) return;
#pragma unroll
            for (int s = 0; s < FP::E; ++s) {
                const int e = ln.t + slot_const<FP, FP::last()>(s);
                if (e < H) gstr(phi, e, v[s].re);
            }
        }
    }
}

template <int N>
struct VacFft {
    template <typename T>
    static hipError_t go(const Launch& L, int64_t pencils, int mode) {
        dim3 grid(unsigned(tiles<N, T>(pencils)), unsigned(L.count));
        const auto b = block<N, T>();
        switch (mode) {
            case kVacZFwd: k_vac_fft<N, T, kVacZFwd><<<grid, b, 0, L.stream>>>(L.members, L.first); break;
            case kVacYFwd: k_vac_fft<N, T, kVacYFwd><<<grid, b, 0, L.stream>>>(L.members, L.first); break;
            case kVacYInv: k_vac_fft<N, T, kVacYInv><<<grid, b, 0, L.stream>>>(L.members, L.first); break;
            default: k_vac_fft<N, T, kVacZInv><<<grid, b, 0, L.stream>>>(L.members, L.first); break;
        }
        return hipGetLastError();
    }
    static hipError_t run(const Launch& L, int prec, int64_t pencils, int mode) {
        return prec ? go<double>(L, pencils, mode) : go<float>(L, pencils, mode);
    }
};

// Spectral kinetic energy: x forward FFT of scratch (already z and y
// transformed) and FP64 partial sums of |k|^2 |psi_k|^2 per work-group.

template <int NY>
struct YFft {
    template <typename T, int V>
    static hipError_t go(const Launch& L, int nx, int nz, bool inv, bool spec) {
        int64_t t;
        if (spec)
            t = tiles<NY, T, V>(int64_t(nx) * (nz / 2)) + tiles<NY, T, V>(nx);
        else
            t = tiles<NY, T, V>(int64_t(nx) * nz);
        dim3 grid(unsigned(t), unsigned(L.count));
        const dim3 b = block<NY, T, V>();
        if (spec) {
            if (inv)
                k_y_fft<NY, T, true, true, V><<<grid, b, 0, L.stream>>>(L.members, L.first);
            else
                k_y_fft<NY, T, false, true, V><<<grid, b, 0, L.stream>>>(L.members, L.first);
        } else {
            if (inv)
                k_y_fft<NY, T, true, false, V><<<grid, b, 0, L.stream>>>(L.members, L.first);
            else
                k_y_fft<NY, T, false, false, V><<<grid, b, 0, L.stream>>>(L.members, L.first);
        }
        return hipGetLastError();
    }
    template <typename T>
    static hipError_t pick(const Launch& L, int nx, int nz, bool inv, bool spec, int var) {
        if constexpr (has_variant(NY))
            if (var == 1) return go<T, 1>(L, nx, nz, inv, spec);
        if constexpr (has_wide(NY)) {
            if (var == 2) return go<T, 2>(L, nx, nz, inv, spec);
            if (var == 3) return go<T, 3>(L, nx, nz, inv, spec);
        }
        return go<T, 0>(L, nx, nz, inv, spec);
    }
    static hipError_t run(const Launch& L, int prec, int nx, int nz, bool inv, bool spec,
                          int var) {
        return prec ? pick<double>(L, nx, nz, inv, spec, var)
                    : pick<float>(L, nx, nz, inv, spec, var);
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

hipError_t launch_y_fft_psi(const Launch& L, int prec, int nx, int ny, int nz, bool inverse,
                            int variant) {
    return dispatch_n<YFft>(ny, L, prec, nx, nz, inverse, false, variant);
}
hipError_t launch_y_fft_spec(const Launch& L, int prec, int nx, int ny, int nz, bool inverse,
                             int variant) {
    return dispatch_n<YFft>(ny, L, prec, nx, nz, inverse, true, variant);
}
hipError_t launch_axis_fft(const Launch& L, int prec, int nx, int ny, int nz, int axis,
                           bool inverse, int which) {
    const int n = axis == 0 ? nx : (axis == 1 ? ny : nz);
    const int64_t pencils = axis == 0 ? int64_t(ny) * nz
                                      : (axis == 1 ? int64_t(nx) * nz : int64_t(nx) * ny);
    return dispatch_n<AxisFft>(n, L, prec, pencils, axis, inverse, which);
}

hipError_t launch_vac_fft(const Launch& L, int prec, int nx, int ny, int nz, int mode) {
    // nx, ny, nz: the padded lengths
    if (mode == kVacZFwd || mode == kVacZInv)
        return dispatch_n<VacFft>(nz, L, prec, int64_t(nx / 2) * (ny / 2), mode);
    return dispatch_n<VacFft>(ny, L, prec, int64_t(nx / 2) * nz, mode);
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
