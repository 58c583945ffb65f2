// Oracle pieces of the learned-corrector workload: shell power spectrum,
// spectral restriction and the 3x3x3 convolution layers (forward and
// backward), all in FP64 straight from their definitions.
#include <cmath>
#include <cstring>

#include "common.hpp"

using namespace orc;

extern "C" {

void orc_power_spectrum(const double* rho, int n, int nbins, double* pk, int64_t* counts) {
    const int64_t N = int64_t(n) * n * n;
    double mean = 0.0;
    for (int64_t i = 0; i < N; ++i) mean += rho[i];
    mean /= double(N);
    std::vector<cplx> f(N);
    for (int64_t i = 0; i < N; ++i) f[i] = cplx(rho[i] / mean - 1.0, 0.0);
    fft3d(f.data(), n, n, n, -1);
    for (int b = 0; b < nbins; ++b) {
        pk[b] = 0.0;
        counts[b] = 0;
    }
    const double norm = 1.0 / (double(N) * double(N));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            for (int64_t k = 0; k < n; ++k) {
                const double mx = double(signed_mode(i, n)), my = double(signed_mode(j, n)),
                             mz = double(signed_mode(k, n));
                const int b = int(std::lround(std::sqrt(mx * mx + my * my + mz * mz)));
                if (b >= nbins) continue;
                pk[b] += std::norm(f[(i * n + j) * n + k]) * norm;
                counts[b] += 1;
            }
    for (int b = 0; b < nbins; ++b)
        if (counts[b] > 0) pk[b] /= double(counts[b]);
}

void orc_restrict(const double* fine_in, int nf, double* coarse_out, int nc) {
    const int64_t Nf = int64_t(nf) * nf * nf, Nc = int64_t(nc) * nc * nc;
    std::vector<cplx> f(reinterpret_cast<const cplx*>(fine_in),
                        reinterpret_cast<const cplx*>(fine_in) + Nf);
    fft3d(f.data(), nf, nf, nf, -1);
    std::vector<cplx> c(Nc, cplx(0.0, 0.0));
    const double scale = double(Nc) / double(Nf);
    for (int64_t i = 0; i < nc; ++i)
        for (int64_t j = 0; j < nc; ++j)
            for (int64_t k = 0; k < nc; ++k) {
                const int64_t m[3] = {signed_mode(i, nc), signed_mode(j, nc), signed_mode(k, nc)};
                bool keep = true;
                for (int a = 0; a < 3; ++a) keep = keep && (m[a] > -nc / 2) && (m[a] < nc / 2);
                if (!keep) continue;
                const int64_t fi = wrap_index(m[0], nf), fj = wrap_index(m[1], nf),
                              fk = wrap_index(m[2], nf);
                c[(i * nc + j) * nc + k] = f[(fi * nf + fj) * nf + fk] * scale;
            }
    fft3d(c.data(), nc, nc, nc, +1);
    std::memcpy(coarse_out, c.data(), sizeof(cplx) * size_t(Nc));
}

static inline int64_t cidx(int64_t i, int64_t j, int64_t k, int64_t n) {
    return (wrap_index(i, n) * n + wrap_index(j, n)) * n + wrap_index(k, n);
}

void orc_conv3d_fwd(const double* x, const double* w, const double* b, double* y, int n, int cin,
                    int cout) {
    const int64_t N = int64_t(n) * n * n;
    parallel_for(int64_t(cout) * n, [&](int64_t b0, int64_t e0) {
        for (int64_t t = b0; t < e0; ++t) {
            const int64_t co = t / n, i = t % n;
            for (int64_t j = 0; j < n; ++j)
                for (int64_t k = 0; k < n; ++k) {
                    double acc = b[co];
                    for (int ci = 0; ci < cin; ++ci)
                        for (int tap = 0; tap < 27; ++tap) {
                            const int ox = tap / 9 - 1, oy = (tap / 3) % 3 - 1, oz = tap % 3 - 1;
                            acc += w[(int64_t(co) * cin + ci) * 27 + tap] *
                                   x[ci * N + cidx(i + ox, j + oy, k + oz, n)];
                        }
                    y[co * N + (i * n + j) * n + k] = acc;
                }
        }
    });
}

void orc_conv3d_bwd(const double* x, const double* w, const double* dy, double* dx, double* dw,
                    double* db, int n, int cin, int cout) {
    const int64_t N = int64_t(n) * n * n;
    // db[co] = sum_p dy[co][p]
    for (int co = 0; co < cout; ++co) {
        double s = 0.0;
        for (int64_t p = 0; p < N; ++p) s += dy[co * N + p];
        db[co] = s;
    }
    // dw[co][ci][tap] = sum_p dy[co][p] x[ci][p + tap]
    parallel_for(int64_t(cout) * cin, [&](int64_t b0, int64_t e0) {
        for (int64_t t = b0; t < e0; ++t) {
            const int64_t co = t / cin, ci = t % cin;
            for (int tap = 0; tap < 27; ++tap) {
                const int ox = tap / 9 - 1, oy = (tap / 3) % 3 - 1, oz = tap % 3 - 1;
                double s = 0.0;
                for (int64_t i = 0; i < n; ++i)
                    for (int64_t j = 0; j < n; ++j)
                        for (int64_t k = 0; k < n; ++k)
                            s += dy[co * N + (i * n + j) * n + k] *
                                 x[ci * N + cidx(i + ox, j + oy, k + oz, n)];
                dw[t * 27 + tap] = s;
            }
        }
    });
    if (!dx) return;
    // dx[ci][q] = sum_{co,tap} w[co][ci][tap] dy[co][q - tap]
    parallel_for(int64_t(cin) * n, [&](int64_t b0, int64_t e0) {
        for (int64_t t = b0; t < e0; ++t) {
            const int64_t ci = t / n, i = t % n;
            for (int64_t j = 0; j < n; ++j)
                for (int64_t k = 0; k < n; ++k) {
                    double s = 0.0;
                    for (int co = 0; co < cout; ++co)
                        for (int tap = 0; tap < 27; ++tap) {
                            const int ox = tap / 9 - 1, oy = (tap / 3) % 3 - 1, oz = tap % 3 - 1;
                            s += w[(int64_t(co) * cin + ci) * 27 + tap] *
                                 dy[co * N + cidx(i - ox, j - oy, k - oz, n)];
                        }
                    dx[ci * N + (i * n + j) * n + k] = s;
                }
        }
    });
}

void orc_round_bf16(double* v, int64_t count) {
    for (int64_t i = 0; i < count; ++i) {
        // float first (round to nearest even), then keep the top 16 bits with
        // round to nearest even on the dropped half.
        float f = float(v[i]);
        uint32_t u;
        std::memcpy(&u, &f, 4);
        if ((u & 0x7f800000u) != 0x7f800000u) {
            const uint32_t lsb = (u >> 16) & 1u;
            u += 0x7fffu + lsb;
        }
        u &= 0xffff0000u;
        std::memcpy(&f, &u, 4);
        v[i] = double(f);
    }
}

}  // extern "C"
