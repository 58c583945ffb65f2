// Internal helpers of the FP64 oracle (test infrastructure only; not shared
// with the GPU library).
#pragma once
#include <algorithm>
#include <complex>
#include <cstdint>
#include <functional>
#include <thread>
#include <vector>

#include "oracle.h"

namespace orc {

using cplx = std::complex<double>;
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kTwoPi = 2.0 * kPi;

int threads();

// Static split of [0, count) over the worker threads.  Every index is handled
// by exactly one call, so results never depend on the number of threads.
void parallel_for(int64_t count, const std::function<void(int64_t, int64_t)>& body);

// Signed FFT index: 0..n/2-1 -> itself, n/2..n-1 -> i - n (Nyquist negative).
inline int64_t signed_mode(int64_t i, int64_t n) { return i < n / 2 ? i : i - n; }

inline int64_t wrap_index(int64_t i, int64_t n) {
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

inline int64_t cells(const orc_config* c) { return int64_t(c->nx) * c->ny * c->nz; }

// Transforms defined in fft.cpp (complex arrays, sign -1 forward / +1 inverse
// with 1/n scaling per axis).
bool fft1d(cplx* x, int n, int sign);
bool fft3d(cplx* d, int nx, int ny, int nz, int sign);

}  // namespace orc
