// Mixed radix-2/3 FFT of the oracle, written from the DFT definition
// X[k] = sum_j x[j] exp(sign * 2 pi i j k / n): decimation in time by 3 while
// 3 divides n, then an iterative radix-2 Cooley-Tukey pass with bit reversal.
// Twiddles are exp(-2 pi i j / n) from std::cos / std::sin, one call per index.
#include <cmath>
#include <map>
#include <mutex>

#include "common.hpp"

namespace orc {

static int g_threads = 0;

int threads() {
    if (g_threads <= 0) {
        unsigned h = std::thread::hardware_concurrency();
        g_threads = h ? int(h) : 1;
    }
    return g_threads;
}

void parallel_for(int64_t count, const std::function<void(int64_t, int64_t)>& body) {
    int nt = threads();
    if (nt <= 1 || count < 2) {
        if (count > 0) body(0, count);
        return;
    }
    nt = int(std::min<int64_t>(nt, count));
    std::vector<std::thread> pool;
    pool.reserve(nt);
    for (int t = 0; t < nt; ++t) {
        int64_t b = count * t / nt, e = count * (t + 1) / nt;
        pool.emplace_back([&body, b, e] { body(b, e); });
    }
    for (auto& th : pool) th.join();
}

// exp(-2 pi i j / n) for j = 0..n-1.
static const std::vector<cplx>& twiddle_table(int n) {
    static std::mutex mu;
    static std::map<int, std::vector<cplx>> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(n);
    if (it != cache.end()) return it->second;
    std::vector<cplx> w(n);
    for (int j = 0; j < n; ++j) {
        double a = -kTwoPi * double(j) / double(n);
        w[j] = cplx(std::cos(a), std::sin(a));
    }
    return cache.emplace(n, std::move(w)).first->second;
}

static bool supported(int n) {
    if (n < 1) return false;
    while (n % 3 == 0) n /= 3;
    while (n % 2 == 0) n /= 2;
    return n == 1;
}

// Unnormalised transform in place; tmp has room for n values.
static void fft_rec(cplx* x, int n, int sign, cplx* tmp) {
    if (n == 1) return;
    const std::vector<cplx>& w = twiddle_table(n);
    auto tw = [&](int64_t e) {
        cplx v = w[size_t(e % n)];
        return sign < 0 ? v : std::conj(v);
    };
    if (n % 3 == 0) {
        // x[3j + r] -> three sub-transforms Y_r, then
        // X[k + m q] = sum_r W^{r (k + m q)} Y_r[k].
        const int m = n / 3;
        for (int r = 0; r < 3; ++r)
            for (int j = 0; j < m; ++j) tmp[r * m + j] = x[3 * j + r];
        for (int r = 0; r < 3; ++r) fft_rec(tmp + r * m, m, sign, x + r * m);
        for (int k = 0; k < m; ++k)
            for (int q = 0; q < 3; ++q) {
                const int kk = k + m * q;
                cplx s = tmp[k];
                s += tw(int64_t(kk)) * tmp[m + k];
                s += tw(int64_t(2) * kk) * tmp[2 * m + k];
                x[kk] = s;
            }
        return;
    }
    // n = 2^a: bit-reversal permutation then log2(n) butterfly sweeps.
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(x[i], x[j]);
    }
    for (int len = 2; len <= n; len <<= 1) {
        const int half = len / 2, step = n / len;
        for (int i = 0; i < n; i += len)
            for (int j = 0; j < half; ++j) {
                cplx u = x[i + j];
                cplx v = x[i + j + half] * tw(int64_t(j) * step);
                x[i + j] = u + v;
                x[i + j + half] = u - v;
            }
    }
}

bool fft1d(cplx* x, int n, int sign) {
    if (!supported(n)) return false;
    std::vector<cplx> tmp(n);
    fft_rec(x, n, sign, tmp.data());
    if (sign > 0) {
        const double s = 1.0 / double(n);
        for (int i = 0; i < n; ++i) x[i] *= s;
    }
    return true;
}

// One axis of a 3D array: pencils of length n with element stride `stride`,
// `count` pencils whose starts are given by start(p).
static void axis_pass(cplx* d, int n, int64_t stride, int64_t count,
                      const std::function<int64_t(int64_t)>& start, int sign) {
    parallel_for(count, [&](int64_t b, int64_t e) {
        std::vector<cplx> line(n), tmp(n);
        for (int64_t p = b; p < e; ++p) {
            cplx* base = d + start(p);
            for (int i = 0; i < n; ++i) line[i] = base[i * stride];
            fft_rec(line.data(), n, sign, tmp.data());
            if (sign > 0) {
                const double s = 1.0 / double(n);
                for (int i = 0; i < n; ++i) line[i] *= s;
            }
            for (int i = 0; i < n; ++i) base[i * stride] = line[i];
        }
    });
}

bool fft3d(cplx* d, int nx, int ny, int nz, int sign) {
    if (!supported(nx) || !supported(ny) || !supported(nz)) return false;
    const int64_t sy = nz, sx = int64_t(ny) * nz;
    // z: contiguous pencils, one per (x, y)
    axis_pass(d, nz, 1, int64_t(nx) * ny, [&](int64_t p) { return p * nz; }, sign);
    // y: pencils per (x, z)
    axis_pass(d, ny, sy, int64_t(nx) * nz,
              [&](int64_t p) { return (p / nz) * sx + (p % nz); }, sign);
    // x: pencils per (y, z)
    axis_pass(d, nx, sx, int64_t(ny) * nz, [&](int64_t p) { return p; }, sign);
    return true;
}

}  // namespace orc

using namespace orc;

extern "C" {

int orc_set_threads(int n) {
    if (n <= 0) {
        unsigned h = std::thread::hardware_concurrency();
        n = h ? int(h) : 1;
    }
    g_threads = n;
    return g_threads;
}

int orc_get_threads(void) { return threads(); }

int orc_fft1d(double* data, int n, int sign) {
    return fft1d(reinterpret_cast<cplx*>(data), n, sign) ? 0 : -1;
}

int orc_fft3d(double* data, int nx, int ny, int nz, int sign) {
    return fft3d(reinterpret_cast<cplx*>(data), nx, ny, nz, sign) ? 0 : -1;
}

void orc_dft3d_brute(const double* in, double* out, int nx, int ny, int nz, int sign) {
    const cplx* x = reinterpret_cast<const cplx*>(in);
    cplx* y = reinterpret_cast<cplx*>(out);
    const int64_t total = int64_t(nx) * ny * nz;
    const double scale = sign > 0 ? 1.0 / double(total) : 1.0;
    parallel_for(total, [&](int64_t b, int64_t e) {
        for (int64_t o = b; o < e; ++o) {
            const int64_t kx = o / (int64_t(ny) * nz), ky = (o / nz) % ny, kz = o % nz;
            cplx acc(0.0, 0.0);
            for (int64_t i = 0; i < total; ++i) {
                const int64_t jx = i / (int64_t(ny) * nz), jy = (i / nz) % ny, jz = i % nz;
                // phase fraction reduced exactly in integers before scaling
                const double frac = double((kx * jx) % nx) / nx + double((ky * jy) % ny) / ny +
                                    double((kz * jz) % nz) / nz;
                const double a = double(sign) * kTwoPi * frac;
                acc += x[i] * cplx(std::cos(a), std::sin(a));
            }
            y[o] = acc * scale;
        }
    });
}

}  // extern "C"
