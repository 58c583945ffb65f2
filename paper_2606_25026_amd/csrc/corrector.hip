// Learned coarse-grid corrector: a three-layer 3x3x3 convolution network
// (3 -> C -> C -> 2 channels, circular padding, ReLU after the hidden layers)
// with BF16 weights and activations on MFMA and FP32 accumulation, its
// backward pass (data and weight gradients, split-K FP32 partials with a
// fixed-order reduction) and Adam.  The network is not part of the paper's
// method; it corrects a 2x-coarser split-step run toward the fine one.
//
// Convolution as an implicit GEMM: out[cell][m] = sum_k W[m][k] in[cell + tap(k)][c(k)]
// with k = tap * CP + c (CP = channels padded to 4 or 16).  One wavefront owns
// 16 cells along z and all 16 (padded) output channels, and issues one
// v_mfma_f32_16x16x16_bf16 per K-chunk of 16:
//   A (16 x 16, M x K): lane l holds W[l % 16][chunk*16 + 4*(l/16) + q], q < 4
//   B (16 x 16, K x N): lane l holds in[cell(l % 16) + tap][c + q] for
//                       k = chunk*16 + 4*(l/16) + q
//   D (16 x 16, M x N): lane l holds out[cell(l % 16)][4*(l/16) + q]
#include "wdm_internal.hpp"

#include <cstdint>

namespace wdm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bf16, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// 4 consecutive bf16 values (8-byte aligned) from global memory
__device__ __forceinline__ bf16x4 ld_bf16x4(const uint16_t* p, int64_t i) {
    return *((const WDM_GAS bf16x4*)(p + i));
}

struct Grid3 {
    int n;   // cubic grid edge
    __device__ __forceinline__ int64_t cells() const { return int64_t(n) * n * n; }
    // neighbour of linear cell p at tap t (offsets (t/9-1, (t/3)%3-1, t%3-1)), periodic
    __device__ __forceinline__ int64_t shift(int64_t p, int t) const {
        const int64_t nn = int64_t(n) * n;
        int x = int(p / nn), y = int((p / n) % n), z = int(p % n);
        x += t / 9 - 1;
        y += (t / 3) % 3 - 1;
        z += t % 3 - 1;
        x = x < 0 ? x + n : (x >= n ? x - n : x);
        y = y < 0 ? y + n : (y >= n ? y - n : y);
        z = z < 0 ? z + n : (z >= n ? z - n : z);
        return (int64_t(x) * n + y) * n + z;
    }
};

// Epilogue modes of the convolution kernel.
enum ConvEpi : int {
    kEpiBiasReluBf16 = 0,   // out = bf16(relu(acc + bias)), CPOUT channels
    kEpiBiasF32 = 1,        // out = f32(acc + bias), COUT channels (network output)
    kEpiMaskBf16 = 2,       // out = bf16(acc * (mask > 0)), CPOUT channels (backward data)
};

// in: bf16 [cells][CPIN]; wmat: bf16 [16][KC*16] (rows >= COUT zero);
// out: see ConvEpi.  COUT real output channels (<= 16), CPOUT padded store width.
template <int CPIN, int COUT, int CPOUT, int EPI>
__global__ __launch_bounds__(256) void k_conv(const uint16_t* __restrict__ in,
                                              const uint16_t* __restrict__ wmat,
                                              const float* __restrict__ bias,
                                              const uint16_t* __restrict__ mask, void* out,
                                              int n) {
    constexpr int KC = (27 * CPIN + 15) / 16;
    const Grid3 g{n};
    const int lane = int(threadIdx.x) & 63;
    const int wave = int(threadIdx.x) >> 6;
    const int64_t seg = int64_t(blockIdx.x) * 4 + wave;      // 16-cell segment along z
    const int64_t base = seg * 16;
    if (base >= g.cells()) return;                            // uniform per wavefront
    const int col = lane & 15;                                // output cell within segment
    const int kq = lane >> 4;                                 // which 4-wide k group
    const int64_t cell = base + col;
    const bool valid = cell < g.cells();   // the last segment may be partial
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 3
    for (int ch = 0; ch < KC; ++ch) {
        const int k0 = ch * 16 + 4 * kq;
        // A: 4 consecutive weights of row (lane % 16)
        const bf16x4 a = ld_bf16x4(wmat, int64_t(col) * (KC * 16) + k0);
        bf16x4 b = {0, 0, 0, 0};
        if (valid && k0 < 27 * CPIN) {
            const int tap = k0 / CPIN, c = k0 % CPIN;
            b = ld_bf16x4(in, g.shift(cell, tap) * CPIN + c);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    if (!valid) return;
    // lane holds out[cell][4*kq + q]
    const int m0 = 4 * kq;
    if constexpr (EPI == kEpiBiasF32) {
        float* o = static_cast<float*>(out);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (m0 + q < COUT) gstr(o, cell * COUT + m0 + q, acc[q] + gldr(bias, m0 + q));
    } else {
        if (m0 >= CPOUT) return;
        uint16_t* o = static_cast<uint16_t*>(out);
        uint16_t r[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float v = acc[q];
            if constexpr (EPI == kEpiBiasReluBf16) {
                v = m0 + q < COUT ? fmaxf(v + gldr(bias, m0 + q), 0.0f) : 0.0f;
            } else {
                const float mk = bf2f(gldr(mask, cell * CPOUT + m0 + q));
                v = (m0 + q < COUT && mk > 0.0f) ? v : 0.0f;
            }
            r[q] = f2bf(v);
        }
        const uint64_t packed = uint64_t(r[0]) | (uint64_t(r[1]) << 16) |
                                (uint64_t(r[2]) << 32) | (uint64_t(r[3]) << 48);
        gstr(reinterpret_cast<uint64_t*>(o), (cell * CPOUT + m0) / 4, packed);
    }
}

// Weight gradient partials.  dz: bf16 [cells][CPZ] (gradient at this layer's
// pre-activation, COUT real channels); act: bf16 [cells][CPIN] (layer input).
// Each work-group sums `chunk` cells and writes
//   part[wg][m][k]  = sum_p dz[p][m] act[p + tap(k)][c(k)]   (m < 16, k < KC*16)
//   part[wg][m][KC*16] = sum_p dz[p][m]                        (bias gradient)
// GEMM roles: M = output channel, N = k, K = cells (16 per MFMA).
template <int CPIN, int CPZ>
__global__ __launch_bounds__(256) void k_conv_wgrad(const uint16_t* __restrict__ dz,
                                                    const uint16_t* __restrict__ act,
                                                    float* __restrict__ part, int n,
                                                    int64_t chunk) {
    constexpr int KC = (27 * CPIN + 15) / 16;
    constexpr int ROW = KC * 16 + 1;
    __shared__ float red[16 * ROW];
    const Grid3 g{n};
    const int lane = int(threadIdx.x) & 63;
    const int wave = int(threadIdx.x) >> 6;
    for (int i = int(threadIdx.x); i < 16 * ROW; i += 256) red[i] = 0.0f;
    __syncthreads();
    f32x4 acc[KC];
#pragma unroll
    for (int t = 0; t < KC; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.0f;
    const int m = lane & 15;      // A row (output channel)
    const int kq = lane >> 4;     // cells 4*kq .. 4*kq+3 of the 16-cell K block
    const int64_t c0 = int64_t(blockIdx.x) * chunk;
    const int64_t c1 = c0 + chunk < g.cells() ? c0 + chunk : g.cells();
    for (int64_t blk = c0 + int64_t(wave) * 16; blk < c1; blk += 64) {
        bf16x4 a;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t p = blk + 4 * kq + q;
            uint16_t v = 0;
            if (p < c1 && m < CPZ) v = gldr(dz, p * CPZ + m);
            a[q] = short(v);
            bsum += bf2f(v);
        }
#pragma unroll
        for (int t = 0; t < KC; ++t) {
            const int k = t * 16 + m;          // B column (lane % 16)
            bf16x4 b = {0, 0, 0, 0};
            if (k < 27 * CPIN) {
                const int tap = k / CPIN, c = k % CPIN;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t p = blk + 4 * kq + q;
                    if (p < c1) b[q] = short(gldr(act, g.shift(p, tap) * CPIN + c));
                }
            }
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
        }
    }
    // D: lane holds [row 4*kq + q][col lane % 16] of every tile; sum the waves in LDS
    // in a fixed order
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int t = 0; t < KC; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) red[(4 * kq + q) * ROW + t * 16 + m] += acc[t][q];
            // bias: lanes with the same m hold partial sums over different cells
            float bs = bsum;
            bs += __shfl_xor(bs, 16);
            bs += __shfl_xor(bs, 32);
            if (kq == 0) red[m * ROW + KC * 16] += bs;
        }
        __syncthreads();
    }
    float* dst = part + int64_t(blockIdx.x) * 16 * ROW;
    for (int i = int(threadIdx.x); i < 16 * ROW; i += 256) gstr(dst, i, red[i]);
}

// Fixed-order sum of the work-group partials: out[i] = sum_b part[b][i].
__global__ void k_sum_partials(const float* __restrict__ part, float* __restrict__ out,
                               int nblocks, int len) {
    const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (i >= len) return;
    float s = 0.0f;
    for (int b = 0; b < nblocks; ++b) s += gldr(part, int64_t(b) * len + i);
    gstr(out, i, s);
}

// ---- packing, loss, Adam ---------------------------------------------------

// f32 [cells][cin] -> bf16 [cells][CP] (zero padded)
__global__ void k_pack_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t cells,
                            int cin, int cp) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= cells * cp) return;
    const int64_t p = i / cp;
    const int c = int(i % cp);
    gstr(y, i, c < cin ? f2bf(gldr(x, p * cin + c)) : uint16_t(0));
}

// loss = sum (y - t)^2 / count in FP64 partials; dy = bf16(2 (y - t) / count)
// stored with CP channels.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             uint16_t* __restrict__ dy, double* __restrict__ part,
                                             int64_t cells, int cout, int cp) {
    __shared__ double red[256];
    const int64_t count = cells * cout;
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < cells * cp;
         i += int64_t(gridDim.x) * 256) {
        const int64_t p = i / cp;
        const int c = int(i % cp);
        float g = 0.0f;
        if (c < cout) {
            const float d = gldr(y, p * cout + c) - gldr(t, p * cout + c);
            s += double(d) * double(d);
            g = float(2.0 * double(d) / double(count));
        }
        gstr(dy, i, f2bf(g));
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) gstr(part, int64_t(blockIdx.x), red[0] / double(count));
}

__global__ void k_sum_f64(const double* __restrict__ part, double* __restrict__ out, int n) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += gldr(part, i);
    gstr(out, 0, s);
}

// Adam on FP32 master parameters (bias-corrected step count t).
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ mo,
                       float* __restrict__ ve, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (i >= n) return;
    const float gi = gldr(g, i);
    const float m = b1 * gldr(mo, i) + (1.0f - b1) * gi;
    const float v = b2 * gldr(ve, i) + (1.0f - b2) * gi * gi;
    gstr(mo, i, m);
    gstr(ve, i, v);
    gstr(w, i, gldr(w, i) - lr * (m / c1) / (sqrtf(v / c2) + eps));
}

// Lay out FP32 weights w[co][ci][27] as the MFMA A matrices:
//   fwd[m][k]  = w[m][c][tap]            k = tap * CPIN + c
//   bwd[m][k]  = w[co][m][26 - tap]      k = tap * CPOUT + co   (transposed, flipped)
__global__ void k_pack_weights(const float* __restrict__ w, uint16_t* __restrict__ fwd,
                               uint16_t* __restrict__ bwd, int cin, int cout, int cpin, int cpout) {
    const int kcf = (27 * cpin + 15) / 16 * 16;
    const int kcb = (27 * cpout + 15) / 16 * 16;
    const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (i < 16 * kcf) {
        const int m = i / kcf, k = i % kcf;
        const int tap = k / cpin, c = k % cpin;
        float v = 0.0f;
        if (m < cout && k < 27 * cpin && c < cin) v = gldr(w, (int64_t(m) * cin + c) * 27 + tap);
        gstr(fwd, i, f2bf(v));
    }
    if (bwd && i < 16 * kcb) {
        const int m = i / kcb, k = i % kcb;
        const int tap = k / cpout, co = k % cpout;
        float v = 0.0f;
        if (m < cin && k < 27 * cpout && co < cout)
            v = gldr(w, (int64_t(co) * cin + m) * 27 + (26 - tap));
        gstr(bwd, i, f2bf(v));
    }
}

// Corrector inputs from a member's state: x[p] = (Re psi * s_psi, Im psi * s_psi,
// Phi * s_phi) as f32 [cells][3].
__global__ void k_state_inputs(const float* __restrict__ psi, const float* __restrict__ phi,
                               float* __restrict__ x, int64_t cells, float s_psi, float s_phi) {
    const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (p >= cells) return;
    gstr(x, 3 * p + 0, gldr(psi, 2 * p) * s_psi);
    gstr(x, 3 * p + 1, gldr(psi, 2 * p + 1) * s_psi);
    gstr(x, 3 * p + 2, gldr(phi, p) * s_phi);
}

// psi += s_out * dpsi (dpsi f32 [cells][2])
__global__ void k_apply_delta(float* __restrict__ psi, const float* __restrict__ d, int64_t cells,
                              float s_out) {
    const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (p >= cells) return;
    gstr(psi, 2 * p, gldr(psi, 2 * p) + s_out * gldr(d, 2 * p));
    gstr(psi, 2 * p + 1, gldr(psi, 2 * p + 1) + s_out * gldr(d, 2 * p + 1));
}

// psi *= sqrt(target / current) with both masses in FP64 (device scalars)
__global__ void k_rescale(float* __restrict__ psi, int64_t cells, const double* __restrict__ before,
                          const double* __restrict__ after) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= 2 * cells) return;
    const double a = gldr(after, 0);
    const float s = a > 0.0 ? float(sqrt(gldr(before, 0) / a)) : 1.0f;
    gstr(psi, i, gldr(psi, i) * s);
}

// FP64 sum of |psi|^2 (partials per block).
__global__ __launch_bounds__(256) void k_mass_partials(const float* __restrict__ psi,
                                                       double* __restrict__ part, int64_t cells) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x; p < cells;
         p += int64_t(gridDim.x) * 256) {
        const double re = gldr(psi, 2 * p), im = gldr(psi, 2 * p + 1);
        s += re * re + im * im;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) gstr(part, int64_t(blockIdx.x), red[0]);
}

// Gradient sums [16][ROW] (k = tap * CPIN + c, bias at column KC*16) to the
// FP32 parameter layout w[co][ci][27], b[co].
__global__ void k_unpack_grads(const float* __restrict__ sum, float* __restrict__ gw,
                               float* __restrict__ gb, int cin, int cout, int cpin, int row) {
    const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
    const int nw = cout * cin * 27;
    if (i < nw) {
        const int co = i / (cin * 27), ci = (i / 27) % cin, tap = i % 27;
        gstr(gw, i, gldr(sum, int64_t(co) * row + tap * cpin + ci));
    } else if (i < nw + cout) {
        const int co = i - nw;
        gstr(gb, co, gldr(sum, int64_t(co) * row + (row - 1)));
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t net_unpack_grads(hipStream_t s, const float* sum, float* gw, float* gb, int cin,
                            int cout, int cpin, int row) {
    const int len = cout * cin * 27 + cout;
    k_unpack_grads<<<(len + 255) / 256, 256, 0, s>>>(sum, gw, gb, cin, cout, cpin, row);
    return hipGetLastError();
}

static unsigned conv_blocks(int n) {
    const int64_t segs = (int64_t(n) * n * n + 15) / 16;
    return unsigned((segs + 3) / 4);
}

hipError_t conv_forward_layer(hipStream_t s, int layer, const uint16_t* in, const uint16_t* w,
                              const float* b, void* out, int n) {
    const unsigned g = conv_blocks(n);
    if (layer == 0)
        k_conv<4, 16, 16, kEpiBiasReluBf16><<<g, 256, 0, s>>>(in, w, b, nullptr, out, n);
    else if (layer == 1)
        k_conv<16, 16, 16, kEpiBiasReluBf16><<<g, 256, 0, s>>>(in, w, b, nullptr, out, n);
    else
        k_conv<16, 2, 4, kEpiBiasF32><<<g, 256, 0, s>>>(in, w, b, nullptr, out, n);
    return hipGetLastError();
}

// Gradient wrt the input of layer `layer` (1 or 2), masked by that input's ReLU.
hipError_t conv_backward_data(hipStream_t s, int layer, const uint16_t* dz, const uint16_t* wbwd,
                              const uint16_t* act_in, uint16_t* dact, int n) {
    const unsigned g = conv_blocks(n);
    if (layer == 2)
        k_conv<4, 16, 16, kEpiMaskBf16><<<g, 256, 0, s>>>(dz, wbwd, nullptr, act_in, dact, n);
    else
        k_conv<16, 16, 16, kEpiMaskBf16><<<g, 256, 0, s>>>(dz, wbwd, nullptr, act_in, dact, n);
    return hipGetLastError();
}

int wgrad_row(int layer) { return ((27 * (layer == 0 ? 4 : 16) + 15) / 16) * 16 + 1; }

hipError_t conv_backward_weight(hipStream_t s, int layer, const uint16_t* dz,
                                const uint16_t* act_in, float* part, int nblocks, float* out,
                                int n) {
    const int64_t cells = int64_t(n) * n * n;
    const int64_t chunk = (cells + nblocks - 1) / nblocks;
    if (layer == 0)
        k_conv_wgrad<4, 16><<<nblocks, 256, 0, s>>>(dz, act_in, part, n, chunk);
    else if (layer == 1)
        k_conv_wgrad<16, 16><<<nblocks, 256, 0, s>>>(dz, act_in, part, n, chunk);
    else
        k_conv_wgrad<16, 4><<<nblocks, 256, 0, s>>>(dz, act_in, part, n, chunk);
    const int len = 16 * wgrad_row(layer);
    k_sum_partials<<<(len + 255) / 256, 256, 0, s>>>(part, out, nblocks, len);
    return hipGetLastError();
}

hipError_t net_pack_input(hipStream_t s, const float* x, uint16_t* y, int64_t cells, int cin,
                          int cp) {
    k_pack_bf16<<<unsigned((cells * cp + 255) / 256), 256, 0, s>>>(x, y, cells, cin, cp);
    return hipGetLastError();
}

hipError_t net_mse(hipStream_t s, const float* y, const float* t, uint16_t* dy, double* part,
                   double* out, int64_t cells, int cout, int cp) {
    constexpr int kBlocks = 1024;
    k_mse<<<kBlocks, 256, 0, s>>>(y, t, dy, part, cells, cout, cp);
    k_sum_f64<<<1, 64, 0, s>>>(part, out, kBlocks);
    return hipGetLastError();
}

hipError_t net_adam(hipStream_t s, float* w, const float* g, float* m, float* v, int n, float lr,
                    float b1, float b2, float eps, float c1, float c2) {
    k_adam<<<(n + 255) / 256, 256, 0, s>>>(w, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t net_pack_weights(hipStream_t s, const float* w, uint16_t* fwd, uint16_t* bwd, int cin,
                            int cout, int cpin, int cpout) {
    const int len = 16 * ((27 * (cpin > cpout ? cpin : cpout) + 15) / 16 * 16);
    k_pack_weights<<<(len + 255) / 256, 256, 0, s>>>(w, fwd, bwd, cin, cout, cpin, cpout);
    return hipGetLastError();
}

hipError_t net_state_inputs(hipStream_t s, const float* psi, const float* phi, float* x,
                            int64_t cells, float s_psi, float s_phi) {
    k_state_inputs<<<unsigned((cells + 255) / 256), 256, 0, s>>>(psi, phi, x, cells, s_psi, s_phi);
    return hipGetLastError();
}

hipError_t net_apply_delta(hipStream_t s, float* psi, const float* d, int64_t cells, float s_out,
                           double* part, double* mass_before, double* mass_after) {
    constexpr int kBlocks = 1024;
    k_mass_partials<<<kBlocks, 256, 0, s>>>(psi, part, cells);
    k_sum_f64<<<1, 64, 0, s>>>(part, mass_before, kBlocks);
    k_apply_delta<<<unsigned((cells + 255) / 256), 256, 0, s>>>(psi, d, cells, s_out);
    k_mass_partials<<<kBlocks, 256, 0, s>>>(psi, part, cells);
    k_sum_f64<<<1, 64, 0, s>>>(part, mass_after, kBlocks);
    k_rescale<<<unsigned((2 * cells + 255) / 256), 256, 0, s>>>(psi, cells, mass_before,
                                                                mass_after);
    return hipGetLastError();
}

}  // namespace wdm
