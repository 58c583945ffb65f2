// FP64 global reductions (mass, potential energy, particle kinetic energy and
// momentum, max |Phi|), the CFL time step of Sec. 3.5, and small utility
// kernels.  Reductions are deterministic: a fixed number of work-groups, each
// summing a fixed range in a fixed order, then one work-group summing the
// partials in order -- no floating-point atomics.
#include <cfloat>

#include "wdm_internal.hpp"
#include "fft_device.hpp"

// wavefront maximum (device library)
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_max_u64(
    unsigned long long);

namespace wdm {

constexpr int kRedThreads = 256;

template <typename T>
__device__ __forceinline__ double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// what 0: sum |psi|^2 -> field 0, max |Phi| -> field 7, max |psi|^2 -> field 8,
//         sum |psi|^4 -> field 9
// what 1: sum (|psi|^2 + scratch) Phi -> field 2 (scratch holds CIC rho_b)
// what 2: sum (|psi|^2 + scratch) Phi_ext -> field 10
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_reduce_grid(const MemberDev* __restrict__ mems,
                                                             int first, int64_t n, int what) {
    __shared__ double red[kRedThreads];
    const MemberDev& m = mems[first];
    const int64_t chunk = (n + kRedBlocks - 1) / kRedBlocks;
    const int64_t b = int64_t(blockIdx.x) * chunk;
    const int64_t e = b + chunk < n ? b + chunk : n;
    const cplx<T>* psi = static_cast<const cplx<T>*>(m.psi);
    const T* phi = static_cast<const T*>(what == 2 ? m.ext : m.phi);
    const T* rb = static_cast<const T*>(m.scratch);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int64_t i = b + threadIdx.x; i < e; i += kRedThreads) {
        const cplx<T> v = gld(psi, i);
        const double re = double(v.re), im = double(v.im);
        const double rho = re * re + im * im;
        if (what == 0) {
            s0 += rho;
            s1 = fmax(s1, fabs(double(gldr(phi, i))));
            s2 = fmax(s2, rho);
            s3 += rho * rho;
        } else {
            s0 += (rho + double(gldr(rb, i))) * double(gldr(phi, i));
        }
    }
    const double t0 = block_sum<T>(s0, red);
    if (what == 0) {
        const double t1 = block_max(s1, red);
        const double t2 = block_max(s2, red);
        const double t3 = block_sum<T>(s3, red);
        if (threadIdx.x == 0) {
            m.partials[int64_t(blockIdx.x) * kRedFields + 0] = t0;
            m.partials[int64_t(blockIdx.x) * kRedFields + 7] = t1;
            m.partials[int64_t(blockIdx.x) * kRedFields + 8] = t2;
            m.partials[int64_t(blockIdx.x) * kRedFields + 9] = t3;
        }
    } else if (threadIdx.x == 0) {
        m.partials[int64_t(blockIdx.x) * kRedFields + (what == 2 ? 10 : 2)] = t0;
    }
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_particles(
    const MemberDev* __restrict__ mems, int first) {
    __shared__ double red[kRedThreads];
    const MemberDev& m = mems[first];
    const int64_t n = m.np;
    const int64_t chunk = (n + kRedBlocks - 1) / kRedBlocks;
    const int64_t b = int64_t(blockIdx.x) * chunk;
    const int64_t e = b + chunk < n ? b + chunk : n;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = b + threadIdx.x; i < e; i += kRedThreads) {
        const double vx = gldr(m.vx, i), vy = gldr(m.vy, i), vz = gldr(m.vz, i);
        s[0] += vx * vx + vy * vy + vz * vz;
        s[1] += vx;
        s[2] += vy;
        s[3] += vz;
    }
    for (int f = 0; f < 4; ++f) {
        const double t = block_sum<float>(s[f], red);
        if (threadIdx.x == 0) m.partials[int64_t(blockIdx.x) * kRedFields + 3 + f] = t;
    }
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_finish(const MemberDev* __restrict__ mems,
                                                               int first, int field, int nblocks,
                                                               int is_max) {
    __shared__ double red[kRedThreads];
    const MemberDev& m = mems[first];
    double s = 0.0;
    for (int i = int(threadIdx.x); i < nblocks; i += kRedThreads) {
        const double v = m.partials[int64_t(i) * kRedFields + field];
        s = is_max ? fmax(s, v) : s + v;
    }
    const double t = is_max ? block_max(s, red) : block_sum<float>(s, red);
    if (threadIdx.x == 0) m.results[field] = t;
}

hipError_t launch_reduce_grid(const Launch& L, int prec, int64_t ncells, int what) {
    if (prec)
        k_reduce_grid<double><<<kRedBlocks, kRedThreads, 0, L.stream>>>(L.members, L.first, ncells,
                                                                        what);
    else
        k_reduce_grid<float><<<kRedBlocks, kRedThreads, 0, L.stream>>>(L.members, L.first, ncells,
                                                                       what);
    return hipGetLastError();
}

hipError_t launch_reduce_particles(const Launch& L, int64_t /*max_np*/) {
    k_reduce_particles<<<kRedBlocks, kRedThreads, 0, L.stream>>>(L.members, L.first);
    return hipGetLastError();
}

hipError_t launch_reduce_finish(const Launch& L, int field, int nblocks, bool is_max) {
    k_reduce_finish<<<1, kRedThreads, 0, L.stream>>>(L.members, L.first, field, nblocks,
                                                     is_max ? 1 : 0);
    return hipGetLastError();
}

// dt = zeta * 0.5 * min{c_kin dx_min^2 / eta, 2 pi eta / max|Phi|,
// 2 pi eta / (|kappa| max|psi|^2)} (Sec. 3.5; the last term only with a
// self-interaction); needs results[7] = max |Phi| and results[8] = max |psi|^2.
// Stored as dt_auto; wdm_step(dt = 0) uses it unless a per-member dt was set.
__global__ void k_dt_auto(const MemberDev* __restrict__ mems, int first, double zeta,
                          double c_kin) {
    const MemberDev& m = mems[first + blockIdx.x];
    const double dx = fmin(m.lx / m.nx, fmin(m.ly / m.ny, m.lz / m.nz));
    double t = c_kin * dx * dx / m.eta;
    const double mp = m.results[7];
    if (mp > 0.0) t = fmin(t, kTwoPi * m.eta / mp);
    const double mr = m.results[8];
    if (m.kappa != 0.0 && mr > 0.0) t = fmin(t, kTwoPi * m.eta / (fabs(m.kappa) * mr));
    m.dt[1] = zeta * 0.5 * t;
}

hipError_t launch_dt_auto(const Launch& L, double zeta, double c_kin) {
    k_dt_auto<<<unsigned(L.count), 1, 0, L.stream>>>(L.members, L.first, zeta, c_kin);
    return hipGetLastError();
}

// Stability check of a wdm_step call (Sec. 3.5): the largest |Phi| (and
// |psi|^2) the call's P1 launches saw give dt_max = 0.5 min{c_kin dx_min^2 /
// eta, 2 pi eta / max|Phi|, 2 pi eta / (|kappa| max|psi|^2)}; stab[0] keeps
// the largest |dt| / dt_max since wdm_set_state, stab[1] is set once a
// non-finite value was seen.
//
// k_watch_fold: many work-groups per member (blockIdx.y) take the maximum of
// their share of the slots, clear it, and fold it into the member's two
// totals after the slots (watch[2 watch_n], watch[2 watch_n + 1]) with an
// integer atomicMax -- max is order-free, so the result is deterministic.
// k_stability then turns the totals into the ratio and clears them.
constexpr int kWatchPerThread = 8;
__global__ __launch_bounds__(256) void k_watch_fold(const MemberDev* __restrict__ mems, int first) {
    __shared__ unsigned long long red[2][4];
    const MemberDev& m = mems[first + blockIdx.y];
    unsigned long long* w = m.watch;
    const int64_t n = m.watch_n;
    unsigned long long a = 0ull, b = 0ull;
    const int64_t base = int64_t(blockIdx.x) * (256 * kWatchPerThread) + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kWatchPerThread; ++k) {
        const int64_t i = base + int64_t(k) * 256;
        if (i < n) {
            a = max(a, w[i]);
            b = max(b, w[n + i]);
            w[i] = 0ull;
            w[n + i] = 0ull;
        }
    }
    a = __ockl_wfred_max_u64(a);
    b = __ockl_wfred_max_u64(b);
    const int wave = int(threadIdx.x) >> 6;
    if (__lane_id() == 0) {
        red[0][wave] = a;
        red[1][wave] = b;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    a = max(max(red[0][0], red[0][1]), max(red[0][2], red[0][3]));
    b = max(max(red[1][0], red[1][1]), max(red[1][2], red[1][3]));
    if (a) atomicMax(w + 2 * n, a);
    if (b) atomicMax(w + 2 * n + 1, b);
}

__global__ void k_stability(const MemberDev* __restrict__ mems, int first, double c_kin) {
    const MemberDev& m = mems[first + blockIdx.x];
    unsigned long long* tot = m.watch + 2 * m.watch_n;
    const double mp = __longlong_as_double((long long)tot[0]);
    const double mr = __longlong_as_double((long long)tot[1]);
    tot[0] = 0ull;
    tot[1] = 0ull;
    if (!(mp <= DBL_MAX) || !(mr <= DBL_MAX)) {
        m.stab[1] = 1.0;
        return;
    }
    const double dx = fmin(m.lx / m.nx, fmin(m.ly / m.ny, m.lz / m.nz));
    double tm = c_kin * dx * dx / m.eta;
    if (mp > 0.0) tm = fmin(tm, kTwoPi * m.eta / mp);
    if (m.kappa != 0.0 && mr > 0.0) tm = fmin(tm, kTwoPi * m.eta / (fabs(m.kappa) * mr));
    m.stab[0] = fmax(m.stab[0], fabs(m.dt[0]) / (0.5 * tm));
}

hipError_t launch_stability(const Launch& L, int64_t slots, double c_kin) {
    const int64_t per = 256 * kWatchPerThread;
    k_watch_fold<<<dim3(unsigned((slots + per - 1) / per), unsigned(L.count)), 256, 0, L.stream>>>(
        L.members, L.first);
    k_stability<<<unsigned(L.count), 1, 0, L.stream>>>(L.members, L.first, c_kin);
    return hipGetLastError();
}

// mode 0: dt in use = dt; 1: dt in use = user dt if set else dt_auto;
// 2: user dt = dt; 3: time = dt
__global__ void k_set_dt(const MemberDev* __restrict__ mems, int first, double dt, int mode) {
    const MemberDev& m = mems[first + blockIdx.x];
    if (mode == 0)
        m.dt[0] = dt;
    else if (mode == 1)
        m.dt[0] = m.dt[2] != 0.0 ? m.dt[2] : m.dt[1];
    else if (mode == 2)
        m.dt[2] = dt;
    else
        m.dt[3] = dt;
}

hipError_t launch_set_dt(const Launch& L, double dt, int mode) {
    k_set_dt<<<unsigned(L.count), 1, 0, L.stream>>>(L.members, L.first, dt, mode);
    return hipGetLastError();
}

// b_a[i] = exp(-alpha dt g_a(i L_a / n_a)) with the face profile of Sec. 3.1,
// g(x) = 2 - tanh(x / w) + tanh((x - L) / w), w = L / n_b, on nodes x in
// [0, L) (the paper centres the box: its x + L/2 is our x).  One work-group
// per member; all ones where alpha dt is 0.
__global__ __launch_bounds__(256) void k_absorb_tables(const MemberDev* __restrict__ mems,
                                                       int first) {
    const MemberDev& m = mems[first + blockIdx.x];
    const double adt = m.absorb_alpha * m.dt[0];
    const int nxy = m.nx + m.ny, n = nxy + m.nz;
    for (int i = int(threadIdx.x); i < n; i += 256) {
        double b = 1.0;
        if (adt != 0.0) {
            const int k = i < m.nx ? i : (i < nxy ? i - m.nx : i - nxy);
            const int len = i < m.nx ? m.nx : (i < nxy ? m.ny : m.nz);
            const double L = i < m.nx ? m.lx : (i < nxy ? m.ly : m.lz);
            const double w = L / m.absorb_nb;
            const double x = double(k) * (L / double(len));
            b = exp(-adt * (2.0 - tanh(x / w) + tanh((x - L) / w)));
        }
        gstr(m.absorb, i, b);
    }
}

hipError_t launch_absorb_tables(const Launch& L) {
    k_absorb_tables<<<unsigned(L.count), 256, 0, L.stream>>>(L.members, L.first);
    return hipGetLastError();
}

__global__ void k_advance_time(const MemberDev* __restrict__ mems, int first, int64_t n) {
    const MemberDev& m = mems[first + blockIdx.x];
    m.dt[3] += double(n) * m.dt[0];
}

hipError_t launch_advance_time(const Launch& L, int64_t nsteps) {
    k_advance_time<<<unsigned(L.count), 1, 0, L.stream>>>(L.members, L.first, nsteps);
    return hipGetLastError();
}

__global__ void k_zero(uint32_t* __restrict__ p, int64_t words) {
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < words;
         i += int64_t(gridDim.x) * 256)
        p[i] = 0u;
}

hipError_t launch_zero(hipStream_t s, void* p, size_t bytes) {
    const int64_t words = int64_t(bytes / 4);
    if (words == 0) return hipSuccess;
    int64_t g = (words + 255) / 256;
    if (g > 8192) g = 8192;
    k_zero<<<unsigned(g), 256, 0, s>>>(static_cast<uint32_t*>(p), words);
    return hipGetLastError();
}

template <typename D, typename S>
__global__ void k_copy_cplx(cplx<D>* __restrict__ dst, const cplx<S>* __restrict__ src, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
        dst[i] = cplx<D>{D(src[i].re), D(src[i].im)};
}

hipError_t launch_copy_complex(hipStream_t s, void* dst, const void* src, int64_t n, int dp,
                               int sp) {
    int64_t g = (n + 255) / 256;
    if (g > 16384) g = 16384;
    if (dp && sp)
        k_copy_cplx<double, double><<<unsigned(g), 256, 0, s>>>(
            static_cast<cplx<double>*>(dst), static_cast<const cplx<double>*>(src), n);
    else if (dp)
        k_copy_cplx<double, float><<<unsigned(g), 256, 0, s>>>(
            static_cast<cplx<double>*>(dst), static_cast<const cplx<float>*>(src), n);
    else if (sp)
        k_copy_cplx<float, double><<<unsigned(g), 256, 0, s>>>(
            static_cast<cplx<float>*>(dst), static_cast<const cplx<double>*>(src), n);
    else
        k_copy_cplx<float, float><<<unsigned(g), 256, 0, s>>>(
            static_cast<cplx<float>*>(dst), static_cast<const cplx<float>*>(src), n);
    return hipGetLastError();
}

template <typename T>
__global__ void k_copy_real(T* __restrict__ dst, const T* __restrict__ src, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
        dst[i] = src[i];
}

hipError_t launch_copy_real(hipStream_t s, void* dst, const void* src, int64_t n, int prec) {
    int64_t g = (n + 255) / 256;
    if (g > 16384) g = 16384;
    if (prec)
        k_copy_real<double><<<unsigned(g), 256, 0, s>>>(static_cast<double*>(dst),
                                                       static_cast<const double*>(src), n);
    else
        k_copy_real<float><<<unsigned(g), 256, 0, s>>>(static_cast<float*>(dst),
                                                      static_cast<const float*>(src), n);
    return hipGetLastError();
}

// rho = |psi|^2 (+ CIC baryon density held in scratch)
template <typename T>
__global__ void k_density_out(const MemberDev* __restrict__ mems, int first, int64_t n,
                              T* __restrict__ out, int inc) {
    const MemberDev& m = mems[first];
    const cplx<T>* psi = static_cast<const cplx<T>*>(m.psi);
    const T* rb = static_cast<const T*>(m.scratch);
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        T r = psi[i].re * psi[i].re + psi[i].im * psi[i].im;
        if (inc) r += rb[i];
        out[i] = r;
    }
}

hipError_t launch_density_out(const Launch& L, int prec, int64_t n, void* out, int inc) {
    int64_t g = (n + 255) / 256;
    if (g > 16384) g = 16384;
    if (prec)
        k_density_out<double><<<unsigned(g), 256, 0, L.stream>>>(L.members, L.first, n,
                                                                static_cast<double*>(out), inc);
    else
        k_density_out<float><<<unsigned(g), 256, 0, L.stream>>>(L.members, L.first, n,
                                                               static_cast<float*>(out), inc);
    return hipGetLastError();
}

template <typename T>
__global__ void k_scale_cplx(cplx<T>* __restrict__ p, int64_t n, T s) {
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
        p[i] = cscale(p[i], s);
}

hipError_t launch_scale_complex(hipStream_t s, void* p, int64_t n, double scale, int prec) {
    int64_t g = (n + 255) / 256;
    if (g > 16384) g = 16384;
    if (prec)
        k_scale_cplx<double><<<unsigned(g), 256, 0, s>>>(static_cast<cplx<double>*>(p), n, scale);
    else
        k_scale_cplx<float><<<unsigned(g), 256, 0, s>>>(static_cast<cplx<float>*>(p), n,
                                                        float(scale));
    return hipGetLastError();
}

// Plain streaming copy: the achievable-bandwidth reference for the roofline.
__global__ __launch_bounds__(256) void k_stream_copy(float4* __restrict__ dst,
                                                     const float4* __restrict__ src, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
        dst[i] = src[i];
}

hipError_t launch_stream_copy(hipStream_t s, float4* dst, const float4* src, int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    k_stream_copy<<<unsigned(g), 256, 0, s>>>(dst, src, n);
    return hipGetLastError();
}

}  // namespace wdm
