// Spectral utilities of the learned-corrector workload: restriction of a fine
// field to a coarser grid (keep the modes the coarse grid resolves, drop its
// Nyquist plane) and the shell power spectrum of the density contrast.
#include "wdm_internal.hpp"
#include "fft_device.hpp"

namespace wdm {

__device__ __forceinline__ int smode(int64_t i, int n) { return int(i < n / 2 ? i : i - n); }

// out[i,j,k] (coarse spectrum, nc^3) = in[m mod nf] * scale for |m_a| < nc/2,
// 0 on the coarse Nyquist planes.
template <typename T>
__global__ void k_restrict_modes(const cplx<T>* __restrict__ fine, cplx<T>* __restrict__ coarse,
                                 int nf, int nc, T scale) {
    const int64_t nc3 = int64_t(nc) * nc * nc;
    for (int64_t o = int64_t(blockIdx.x) * 256 + threadIdx.x; o < nc3;
         o += int64_t(gridDim.x) * 256) {
        const int mi = smode(o / (int64_t(nc) * nc), nc);
        const int mj = smode((o / nc) % nc, nc);
        const int mk = smode(o % nc, nc);
        cplx<T> v{T(0), T(0)};
        if (mi != -nc / 2 && mj != -nc / 2 && mk != -nc / 2) {
            const int64_t fi = mi < 0 ? mi + nf : mi, fj = mj < 0 ? mj + nf : mj,
                          fk = mk < 0 ? mk + nf : mk;
            v = cscale(gld(fine, (fi * nf + fj) * nf + fk), scale);
        }
        gst(coarse, o, v);
    }
}

hipError_t launch_restrict_modes(hipStream_t s, const void* fine, void* coarse, int nf, int nc,
                                 int prec) {
    const int64_t nc3 = int64_t(nc) * nc * nc;
    int64_t g = (nc3 + 255) / 256;
    if (g > 16384) g = 16384;
    const double scale = 1.0 / (double(nf) * nf * nf);
    if (prec)
        k_restrict_modes<double><<<unsigned(g), 256, 0, s>>>(
            static_cast<const cplx<double>*>(fine), static_cast<cplx<double>*>(coarse), nf, nc,
            scale);
    else
        k_restrict_modes<float><<<unsigned(g), 256, 0, s>>>(
            static_cast<const cplx<float>*>(fine), static_cast<cplx<float>*>(coarse), nf, nc,
            float(scale));
    return hipGetLastError();
}

// scratch = (|psi|^2 N / sum|psi|^2 - 1, 0); the FP64 sum is results[0].
template <typename T>
__global__ void k_contrast(const MemberDev* __restrict__ mems, int first, int64_t n) {
    const MemberDev& m = mems[first];
    const double mean = gldr(m.results, 0) / double(n);
    const cplx<T>* psi = static_cast<const cplx<T>*>(m.psi);
    cplx<T>* out = static_cast<cplx<T>*>(m.scratch);
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        const cplx<T> v = gld(psi, i);
        const double r = double(v.re) * v.re + double(v.im) * v.im;
        gst(out, i, cplx<T>{T(r / mean - 1.0), T(0)});
    }
}

hipError_t launch_contrast(const Launch& L, int prec, int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 16384) g = 16384;
    if (prec)
        k_contrast<double><<<unsigned(g), 256, 0, L.stream>>>(L.members, L.first, n);
    else
        k_contrast<float><<<unsigned(g), 256, 0, L.stream>>>(L.members, L.first, n);
    return hipGetLastError();
}

// Shell sums of |delta_k|^2 / N^2 over b = round(|m|) < nbins (cubic grid);
// each block writes part[block][0..nbins) sums and [nbins..2 nbins) counts.
constexpr int kPkBlocks = 64;
constexpr int kPkMaxBins = 1024;

template <typename T>
__global__ __launch_bounds__(256) void k_shells(const MemberDev* __restrict__ mems, int first,
                                                int nbins, double* __restrict__ part) {
    __shared__ double sum[kPkMaxBins];
    __shared__ unsigned long long cnt[kPkMaxBins];
    const MemberDev& m = mems[first];
    for (int b = int(threadIdx.x); b < nbins; b += 256) {
        sum[b] = 0.0;
        cnt[b] = 0ull;
    }
    __syncthreads();
    const int n = m.nx;
    const int64_t N = int64_t(n) * n * n;
    const double norm = 1.0 / (double(N) * double(N));
    const cplx<T>* f = static_cast<const cplx<T>*>(m.scratch);
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < N;
         i += int64_t(gridDim.x) * 256) {
        const double mx = smode(i / (int64_t(n) * n), n), my = smode((i / n) % n, n),
                     mz = smode(i % n, n);
        const int b = int(rint(sqrt(mx * mx + my * my + mz * mz)));
        if (b >= nbins) continue;
        const cplx<T> v = gld(f, i);
        atomicAdd(&sum[b], (double(v.re) * v.re + double(v.im) * v.im) * norm);
        atomicAdd(&cnt[b], 1ull);
    }
    __syncthreads();
    for (int b = int(threadIdx.x); b < nbins; b += 256) {
        gstr(part, int64_t(blockIdx.x) * 2 * nbins + b, sum[b]);
        gstr(part, int64_t(blockIdx.x) * 2 * nbins + nbins + b, double(cnt[b]));
    }
}

__global__ void k_shells_finish(const double* __restrict__ part, double* __restrict__ out,
                                int nbins, int nblocks) {
    const int b = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (b >= 2 * nbins) return;
    double s = 0.0;
    for (int k = 0; k < nblocks; ++k) s += gldr(part, int64_t(k) * 2 * nbins + b);
    gstr(out, b, s);
}

hipError_t launch_shells(const Launch& L, int prec, int nbins, double* part, double* out) {
    if (nbins < 1 || nbins > kPkMaxBins) return hipErrorInvalidValue;
    if (prec)
        k_shells<double><<<kPkBlocks, 256, 0, L.stream>>>(L.members, L.first, nbins, part);
    else
        k_shells<float><<<kPkBlocks, 256, 0, L.stream>>>(L.members, L.first, nbins, part);
    k_shells_finish<<<(2 * nbins + 255) / 256, 256, 0, L.stream>>>(part, out, nbins, kPkBlocks);
    return hipGetLastError();
}

size_t shells_partial_doubles() { return size_t(kPkBlocks) * 2 * kPkMaxBins + 2 * kPkMaxBins; }

// FP64 partials of sum |psi - other|^2 and sum |other|^2 (the judge's field
// distance) into part[2 b], part[2 b + 1] over a fixed grid of work-groups,
// then their ordered sums into out[0], out[1].
constexpr int kDistBlocks = 1024;

template <typename T>
__global__ __launch_bounds__(256) void k_distance(const MemberDev* __restrict__ mems, int first,
                                                  const cplx<T>* __restrict__ other, int64_t n,
                                                  double* __restrict__ part) {
    __shared__ double red[2][256];
    const MemberDev& m = mems[first];
    const cplx<T>* psi = static_cast<const cplx<T>*>(m.psi);
    double d = 0.0, o = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        const cplx<T> a = gld(psi, i), b = gld(other, i);
        const double dr = double(a.re) - double(b.re), di = double(a.im) - double(b.im);
        d += dr * dr + di * di;
        o += double(b.re) * double(b.re) + double(b.im) * double(b.im);
    }
    red[0][threadIdx.x] = d;
    red[1][threadIdx.x] = o;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        gstr(part, 2 * int64_t(blockIdx.x), red[0][0]);
        gstr(part, 2 * int64_t(blockIdx.x) + 1, red[1][0]);
    }
}

// The two sums of the kDistBlocks partial pairs in a fixed order (thread t
// adds blocks t, t + 256, ..., then the work-group tree).
__global__ __launch_bounds__(256) void k_distance_finish(const double* __restrict__ part,
                                                         double* __restrict__ out) {
    __shared__ double red[2][256];
    const int t = int(threadIdx.x);
    double d = 0.0, o = 0.0;
    for (int b = t; b < kDistBlocks; b += 256) {
        d += gldr(part, 2 * b);
        o += gldr(part, 2 * b + 1);
    }
    red[0][t] = d;
    red[1][t] = o;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            red[0][t] += red[0][t + w];
            red[1][t] += red[1][t + w];
        }
        __syncthreads();
    }
    if (t != 0) return;
    gstr(out, 0, red[0][0]);
    gstr(out, 1, red[1][0]);
}

hipError_t launch_distance(const Launch& L, int prec, const void* other, int64_t n, double* part,
                           double* out) {
    if (prec)
        k_distance<double><<<kDistBlocks, 256, 0, L.stream>>>(
            L.members, L.first, static_cast<const cplx<double>*>(other), n, part);
    else
        k_distance<float><<<kDistBlocks, 256, 0, L.stream>>>(
            L.members, L.first, static_cast<const cplx<float>*>(other), n, part);
    k_distance_finish<<<1, 256, 0, L.stream>>>(part, out);
    return hipGetLastError();
}

}  // namespace wdm
