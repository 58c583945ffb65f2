// Diagnostics of a synchronised state (Sec. 3.6, App. A.1): the paper's
// overall energy terms K, Q, V with the wave momentum, and the radii that
// enclose fixed fractions of the wave mass around a centre node.
#include "wdm_internal.hpp"
#include "fft_device.hpp"

namespace wdm {

constexpr int kDiagThreads = 256;
constexpr int kDiagFields = 7;   // K, Q, V, Px, Py, Pz, sum |psi|^2 (each times 1/dV)

__device__ __forceinline__ double diag_block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kDiagThreads / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Per cell, second-order central differences on the periodic nodes:
//   j_a = eta Im(psi* (psi_{+a} - psi_{-a}) / (2 h_a))   (momentum density rho v),
//   K += j.j / (2 rho) for rho > 1e-30,  Q += sum_a ((|psi_{+a}| - |psi_{-a}|) / (2 h_a))^2,
//   V += rho Phi,  P += j,  M += rho.
// Each work-group sums a fixed range in a fixed order (deterministic); the
// partials go to fields 0..6 and are finished by k_reduce_finish.
template <typename T>
__global__ __launch_bounds__(kDiagThreads) void k_diag_energies(const MemberDev* __restrict__ mems,
                                                                int first, int nblocks) {
    __shared__ double red[kDiagThreads];
    const MemberDev& m = mems[first];
    const int64_t nyz = int64_t(m.ny) * m.nz, n = int64_t(m.nx) * nyz;
    const int64_t chunk = (n + nblocks - 1) / nblocks;
    const int64_t b = int64_t(blockIdx.x) * chunk;
    const int64_t e = b + chunk < n ? b + chunk : n;
    const cplx<T>* psi = static_cast<const cplx<T>*>(m.psi);
    const T* phi = static_cast<const T*>(m.phi);
    const double inv2h[3] = {0.5 * m.inv_dx, 0.5 * m.inv_dy, 0.5 * m.inv_dz};
    double acc[kDiagFields] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = b + threadIdx.x; i < e; i += kDiagThreads) {
        const int64_t ix = i / nyz, r = i - ix * nyz;
        const int iy = int(r / m.nz), iz = int(r - int64_t(iy) * m.nz);
        const int64_t xp = (ix + 1 == m.nx ? 0 : ix + 1) * nyz + r;
        const int64_t xm = (ix == 0 ? m.nx - 1 : ix - 1) * nyz + r;
        const int64_t row = ix * nyz + iz;
        const int64_t yp = row + int64_t(iy + 1 == m.ny ? 0 : iy + 1) * m.nz;
        const int64_t ym = row + int64_t(iy == 0 ? m.ny - 1 : iy - 1) * m.nz;
        const int64_t zrow = i - iz;
        const int64_t zp = zrow + (iz + 1 == m.nz ? 0 : iz + 1);
        const int64_t zm = zrow + (iz == 0 ? m.nz - 1 : iz - 1);
        const int64_t nb[3][2] = {{xp, xm}, {yp, ym}, {zp, zm}};
        const cplx<T> c = gld(psi, i);
        const double cr = double(c.re), ci = double(c.im);
        const double rho = cr * cr + ci * ci;
        double j2 = 0.0, q2 = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const cplx<T> p = gld(psi, nb[a][0]), q = gld(psi, nb[a][1]);
            const double dre = (double(p.re) - double(q.re)) * inv2h[a];
            const double dim = (double(p.im) - double(q.im)) * inv2h[a];
            const double ja = m.eta * (cr * dim - ci * dre);
            j2 += ja * ja;
            acc[3 + a] += ja;
            const double ap = sqrt(double(p.re) * double(p.re) + double(p.im) * double(p.im));
            const double aq = sqrt(double(q.re) * double(q.re) + double(q.im) * double(q.im));
            const double ds = (ap - aq) * inv2h[a];
            q2 += ds * ds;
        }
        if (rho > 1e-30) acc[0] += 0.5 * j2 / rho;
        acc[1] += q2;
        acc[2] += rho * double(gldr(phi, i));
        acc[6] += rho;
    }
    for (int f = 0; f < kDiagFields; ++f) {
        const double t = diag_block_sum(acc[f], red);
        if (threadIdx.x == 0) m.partials[int64_t(blockIdx.x) * kRedFields + f] = t;
    }
}

// Wave mass per squared node distance s = di^2 + dj^2 + dk^2 (minimum-image
// offsets from the centre node; cubic cells), accumulated with FP64 atomics
// into hist[0..smax] (cleared by the caller).
template <typename T>
__global__ __launch_bounds__(256) void k_radial_hist(const MemberDev* __restrict__ mems, int first,
                                                     int ci, int cj, int ck,
                                                     double* __restrict__ hist) {
    const MemberDev& m = mems[first];
    const int64_t nyz = int64_t(m.ny) * m.nz, n = int64_t(m.nx) * nyz;
    const cplx<T>* psi = static_cast<const cplx<T>*>(m.psi);
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        const int64_t ix = i / nyz, r = i - ix * nyz;
        const int iy = int(r / m.nz), iz = int(r - int64_t(iy) * m.nz);
        int di = int(ix) - ci, dj = iy - cj, dk = iz - ck;
        di = di < 0 ? -di : di;
        dj = dj < 0 ? -dj : dj;
        dk = dk < 0 ? -dk : dk;
        di = di > m.nx - di ? m.nx - di : di;
        dj = dj > m.ny - dj ? m.ny - dj : dj;
        dk = dk > m.nz - dk ? m.nz - dk : dk;
        const cplx<T> v = gld(psi, i);
        const double rho = double(v.re) * double(v.re) + double(v.im) * double(v.im);
        if (rho != 0.0) gatomic_add(hist + (di * di + dj * dj + dk * dk), rho);
    }
}

// One work-group: running sums of hist[0..nbins) and, for f = 0.1, ..., 0.9,
// the first non-empty bin s whose running sum reaches f times the total;
// out[f] = dx sqrt(s).
__global__ __launch_bounds__(256) void k_mass_radii(const double* __restrict__ hist,
                                                    int64_t nbins, double dx,
                                                    double* __restrict__ out) {
    __shared__ double part[256];
    __shared__ double base[257];
    __shared__ unsigned long long first_bin;
    const int t = int(threadIdx.x);
    const int64_t chunk = (nbins + 255) / 256;
    const int64_t b = t * chunk, e = b + chunk < nbins ? b + chunk : nbins;
    double s = 0.0;
    for (int64_t k = b; k < e; ++k) s += hist[k];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        base[0] = 0.0;
        for (int u = 0; u < 256; ++u) base[u + 1] = base[u] + part[u];
    }
    __syncthreads();
    const double total = base[256];
    for (int f = 1; f <= 9; ++f) {
        const double thr = 0.1 * double(f) * total;
        if (t == 0) first_bin = (unsigned long long)nbins;
        __syncthreads();
        double cum = base[t];
        for (int64_t k = b; k < e; ++k) {
            cum += hist[k];
            if (hist[k] > 0.0 && cum >= thr) {
                atomicMin(&first_bin, (unsigned long long)k);
                break;
            }
        }
        __syncthreads();
        if (t == 0)
            out[f - 1] = first_bin < (unsigned long long)nbins ? dx * sqrt(double(first_bin)) : -1.0;
        __syncthreads();
    }
}

hipError_t launch_diag_energies(const Launch& L, int prec, int nblocks) {
    if (prec)
        k_diag_energies<double><<<nblocks, kDiagThreads, 0, L.stream>>>(L.members, L.first,
                                                                         nblocks);
    else
        k_diag_energies<float><<<nblocks, kDiagThreads, 0, L.stream>>>(L.members, L.first,
                                                                        nblocks);
    return hipGetLastError();
}

hipError_t launch_mass_radii(const Launch& L, int prec, int64_t ncells, const int centre[3],
                             double dx, double* hist, int64_t nbins, double* out) {
    hipError_t e = launch_zero(L.stream, hist, size_t(nbins) * sizeof(double));
    if (e != hipSuccess) return e;
    int64_t g = (ncells + 255) / 256;
    if (g > 4096) g = 4096;
    if (prec)
        k_radial_hist<double><<<unsigned(g), 256, 0, L.stream>>>(L.members, L.first, centre[0],
                                                                 centre[1], centre[2], hist);
    else
        k_radial_hist<float><<<unsigned(g), 256, 0, L.stream>>>(L.members, L.first, centre[0],
                                                                centre[1], centre[2], hist);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_mass_radii<<<1, 256, 0, L.stream>>>(hist, nbins, dx, out);
    return hipGetLastError();
}

}  // namespace wdm
