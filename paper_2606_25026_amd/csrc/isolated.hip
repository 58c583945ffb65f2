// Vacuum-boundary Poisson solve (Sec. 3.2.1) and the external tidal potential
// (Sec. 4.3).
//
// The isolated potential is the linear convolution of the density with the
// free-space Green's function, done as a circular convolution on the grid
// zero-padded to (2 nx, 2 ny, 2 nz): the density, in the padded grid's corner,
// is transformed, multiplied by the transform of the padded Green's function
// (real and even, computed once per plan) and transformed back; the corner is
// the potential.  The transforms (passes_y.hip, launch_vac_fft, and the x pass
// here, which multiplies by the Green's function between its forward and
// inverse transforms) run on the padded grid through a second member table
// whose entries describe it, and touch only the parts of it that can be
// non-zero.
#include "wdm_internal.hpp"
#include "fft_device.hpp"

namespace wdm {

constexpr int kIsoThreads = 256;
typedef float wdm_f4v __attribute__((ext_vector_type(4)));

static unsigned iso_grid(int64_t count) {
    int64_t g = (count + kIsoThreads - 1) / kIsoThreads;
    return unsigned(g < 8192 ? g : 8192);
}

// g = -G dV / |r| between nodes, -G h^2 C for the node itself (cubic cells of
// side h; C = 6 ln((1 + sqrt 3) / sqrt 2) - pi / 2, the integral of 1/|u| over
// the unit cube centred at 0), with the offsets of the padded circulant
// (index i and i - 2n are the same offset).
template <typename T>
__global__ __launch_bounds__(kIsoThreads) void k_green_fill(const MemberDev* __restrict__ mems,
                                                            int first) {
    const MemberDev& m = mems[first + blockIdx.y];
    const int64_t px = 2 * int64_t(m.nx), py = 2 * int64_t(m.ny), pz = 2 * int64_t(m.nz);
    const int64_t total = px * py * pz;
    const double G = m.four_pi_G / (4.0 * kPi);
    const double h = m.lx / m.nx, dv = h * h * h;
    const double C = 6.0 * log((1.0 + sqrt(3.0)) / sqrt(2.0)) - 0.5 * kPi;
    cplx<T>* pad = static_cast<cplx<T>*>(m.pad);
    for (int64_t q = int64_t(blockIdx.x) * kIsoThreads + threadIdx.x; q < total;
         q += int64_t(gridDim.x) * kIsoThreads) {
        const int64_t i = q / (py * pz), r = q - i * py * pz;
        const int64_t j = r / pz, k = r - j * pz;
        const int64_t di = i <= m.nx ? i : i - px, dj = j <= m.ny ? j : j - py,
                      dk = k <= m.nz ? k : k - pz;
        double g;
        if (di == 0 && dj == 0 && dk == 0) {
            g = -G * h * h * C;
        } else {
            const double x = double(di) * h, y = double(dj) * h, z = double(dk) * h;
            g = -G * dv / sqrt(x * x + y * y + z * z);
        }
        gst(pad, q, cplx<T>{T(g), T(0)});
    }
}

// The step's transforms are unnormalised in both directions: the padded round
// trip and the z round trip through the half spectrum (into P1) multiply by
// 8 nx ny nz and by nz; both factors are taken out here, once.  The padded
// kernel is even along each axis (g[i] = g[2n - i]), so its transform is real
// and even along each axis: only modes 0..n of each axis are kept, a
// (nx + 1)(ny + 1)(nz + 1) table, and mode k > n reads mode 2n - k.
template <typename T>
__global__ __launch_bounds__(kIsoThreads) void k_green_extract(const MemberDev* __restrict__ mems,
                                                               int first) {
    const MemberDev& m = mems[first + blockIdx.y];
    const int64_t fy = m.ny + 1, fz = m.nz + 1;
    const int64_t total = (m.nx + 1) * fy * fz;
    const int64_t py = 2 * int64_t(m.ny), pz = 2 * int64_t(m.nz);
    const double scale = 1.0 / (8.0 * double(m.nx) * m.ny * m.nz * double(m.nz));
    const cplx<T>* pad = static_cast<const cplx<T>*>(m.pad);
    T* green = static_cast<T*>(m.green);
    for (int64_t q = int64_t(blockIdx.x) * kIsoThreads + threadIdx.x; q < total;
         q += int64_t(gridDim.x) * kIsoThreads) {
        const int64_t i = q / (fy * fz), r = q - i * fy * fz;
        const int64_t j = r / fz, k = r - j * fz;
        gstr(green, q, T(double(gld(pad, (i * py + j) * pz + k).re) * scale));
    }
}


// Mean gradient of ext along each axis over the nodes symmetric about the
// centre node: sums of (ext[n-1] - ext[1]) over the other two axes, per
// work-group in a fixed range and order (fields 0..2), finished by
// k_reduce_finish.
template <typename T>
__global__ __launch_bounds__(kIsoThreads) void k_tidal_partials(const MemberDev* __restrict__ mems,
                                                                int first, int nblocks) {
    __shared__ double red[kIsoThreads];
    const MemberDev& m = mems[first];
    const int64_t nyz = int64_t(m.ny) * m.nz, n = int64_t(m.nx) * nyz;
    const int64_t chunk = (n + nblocks - 1) / nblocks;
    const int64_t b = int64_t(blockIdx.x) * chunk;
    const int64_t e = b + chunk < n ? b + chunk : n;
    const T* ext = static_cast<const T*>(m.ext);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t c = b + threadIdx.x; c < e; c += kIsoThreads) {
        const int64_t i = c / nyz, r = c - i * nyz;
        const int64_t j = r / m.nz, k = r - j * m.nz;
        const double v = double(gldr(ext, c));
        if (i == m.nx - 1) acc[0] += v - double(gldr(ext, (1 * m.ny + j) * m.nz + k));
        if (j == m.ny - 1) acc[1] += v - double(gldr(ext, (i * m.ny + 1) * m.nz + k));
        if (k == m.nz - 1) acc[2] += v - double(gldr(ext, (i * m.ny + j) * m.nz + 1));
    }
    for (int a = 0; a < 3; ++a) {
        red[threadIdx.x] = acc[a];
        __syncthreads();
        for (int w = kIsoThreads / 2; w > 0; w >>= 1) {
            if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) m.partials[int64_t(blockIdx.x) * kRedFields + a] = red[0];
        __syncthreads();
    }
}

// ext -= sum_a g_a (x_a - L_a / 2), g_a = S_a / ((n_b n_c) (n_a - 2) h_a).
template <typename T>
__global__ __launch_bounds__(kIsoThreads) void k_tidal_apply(const MemberDev* __restrict__ mems,
                                                             int first) {
    const MemberDev& m = mems[first];
    const int64_t nyz = int64_t(m.ny) * m.nz, n = int64_t(m.nx) * nyz;
    const double h[3] = {m.lx / m.nx, m.ly / m.ny, m.lz / m.nz};
    const double cnt[3] = {double(nyz), double(int64_t(m.nx) * m.nz), double(int64_t(m.nx) * m.ny)};
    const int len[3] = {m.nx, m.ny, m.nz};
    double g[3];
    for (int a = 0; a < 3; ++a) g[a] = m.results[a] / cnt[a] / (double(len[a] - 2) * h[a]);
    T* ext = static_cast<T*>(m.ext);
    for (int64_t c = int64_t(blockIdx.x) * kIsoThreads + threadIdx.x; c < n;
         c += int64_t(gridDim.x) * kIsoThreads) {
        const int64_t i = c / nyz, r = c - i * nyz;
        const int64_t j = r / m.nz, k = r - j * m.nz;
        const double x = double(i) * h[0] - 0.5 * m.lx, y = double(j) * h[1] - 0.5 * m.ly,
                     z = double(k) * h[2] - 0.5 * m.lz;
        gstr(ext, c, T(double(gldr(ext, c)) - g[0] * x - g[1] * y - g[2] * z));
    }
}

#define WDM_ISO_LAUNCH(KERNEL, COUNT)                                                      \
    do {                                                                                   \
        const dim3 grid(iso_grid(COUNT), unsigned(L.count));                               \
        if (prec)                                                                          \
            KERNEL<double><<<grid, kIsoThreads, 0, L.stream>>>(L.members, L.first);        \
        else                                                                               \
            KERNEL<float><<<grid, kIsoThreads, 0, L.stream>>>(L.members, L.first);         \
        return hipGetLastError();                                                          \
    } while (0)

hipError_t launch_green_fill(const Launch& L, int prec, int64_t max_cells) {
    WDM_ISO_LAUNCH(k_green_fill, 8 * max_cells);
}
hipError_t launch_green_extract(const Launch& L, int prec, int64_t max_cells) {
    WDM_ISO_LAUNCH(k_green_extract, 8 * max_cells);
}
#undef WDM_ISO_LAUNCH

hipError_t launch_tidal_correct(const Launch& L, int prec, int64_t ncells) {
    hipError_t e;
    if (prec)
        k_tidal_partials<double><<<kRedBlocks, kIsoThreads, 0, L.stream>>>(L.members, L.first,
                                                                           kRedBlocks);
    else
        k_tidal_partials<float><<<kRedBlocks, kIsoThreads, 0, L.stream>>>(L.members, L.first,
                                                                          kRedBlocks);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int a = 0; a < 3; ++a)
        if ((e = launch_reduce_finish(L, a, kRedBlocks, false)) != hipSuccess) return e;
    if (prec)
        k_tidal_apply<double><<<iso_grid(ncells), kIsoThreads, 0, L.stream>>>(L.members, L.first);
    else
        k_tidal_apply<float><<<iso_grid(ncells), kIsoThreads, 0, L.stream>>>(L.members, L.first);
    return hipGetLastError();
}

}  // namespace wdm
