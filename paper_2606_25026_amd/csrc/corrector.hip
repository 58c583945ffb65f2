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
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
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
    // the correction (COUT = 2): out is psi (f32 re, im per cell),
    // psi += s_out (acc + bias) with s_out = scal[5], and part[work-group] gets
    // the FP64 sum of the corrected |psi|^2 over the work-group's cells
    kEpiApply = 3,
};

// Convolution tile: 4 x 4 x 16 output cells (x, y, z) per work-group pass.
// The input brick with its one-cell periodic halo, 6 x 6 x 18 cells, is staged
// in LDS once and read by all 27 taps; each wavefront owns the four 16-cell z
// segments of one x row (N = 16 cells per MFMA) and keeps its A operand (the
// layer's weights, all K chunks) in registers for the whole launch.
constexpr int kCTX = 4, kCTY = 4, kCTZ = 16;
constexpr int kCBX = kCTX + 2, kCBY = kCTY + 2, kCBZ = kCTZ + 2;
constexpr int kCBrick = kCBX * kCBY * kCBZ;

// v in [-1, n + kCTZ]: periodic index in [0, n)
__device__ __forceinline__ int wrap_edge(int v, int n) { return (v + n) % n; }

// The input brick of tile t: every 8-byte word of its cells (one 16-byte half
// cell per thread and slot for 16 channels, one 8-byte cell for 4), loaded into
// registers; stored to LDS by brick_store.
template <int W8>
struct BrickRegs {
    static constexpr int kWords = kCBrick * W8;              // 8-byte words
    static constexpr int kPer = W8 == 4 ? 2 : 1;             // words per load
    static constexpr int kLoads = kWords / kPer;
    static constexpr int kIt = (kLoads + 255) / 256;
    u32x4 v[W8 == 4 ? kIt : 1];
    uint64_t w[W8 == 4 ? 1 : kIt];
};

template <int CPIN, int W8>
__device__ __forceinline__ void brick_load(BrickRegs<W8>& R, const uint16_t* __restrict__ in,
                                           int64_t t, int n, int tz, int ty) {
    using B = BrickRegs<W8>;
    const int tid = int(threadIdx.x);
    const int iz = int(t % tz);
    const int64_t r = t / tz;
    const int x0 = int(r / ty) * kCTX, y0 = int(r % ty) * kCTY, z0 = iz * kCTZ;
#pragma unroll
    for (int k = 0; k < B::kIt; ++k) {
        const int i = tid + k * 256;
        if (i < B::kLoads) {
            const int c = i / (W8 / B::kPer), bz = c % kCBZ, rr = c / kCBZ, by = rr % kCBY,
                      bx = rr / kCBY;
            const int64_t g = (int64_t(wrap_edge(x0 + bx - 1, n)) * n +
                               wrap_edge(y0 + by - 1, n)) * n + wrap_edge(z0 + bz - 1, n);
            if constexpr (W8 == 4)
                R.v[k] = *(const WDM_GAS u32x4*)(in + g * CPIN + (i & 1) * 8);
            else
                R.w[k] = *(const WDM_GAS uint64_t*)(in + g * CPIN);
        }
    }
}

template <int W8>
__device__ __forceinline__ void brick_store(const BrickRegs<W8>& R, uint64_t* brick) {
    using B = BrickRegs<W8>;
    const int tid = int(threadIdx.x);
#pragma unroll
    for (int k = 0; k < B::kIt; ++k) {
        const int i = tid + k * 256;
        if (i < B::kLoads) {
            if constexpr (W8 == 4)
                reinterpret_cast<u32x4*>(brick)[i] = R.v[k];
            else
                brick[i] = R.w[k];
        }
    }
}

// in: bf16 [cells][CPIN]; wmat: bf16 [16][KC*16] (rows >= COUT zero);
// out: see ConvEpi.  COUT real output channels (<= 16), CPOUT padded store width.
// Persistent: work-group b handles tiles b, b + gridDim.x, ...; the next
// tile's brick is loaded into registers while the current one is computed.
// The layer's weights (the MFMA A operand) sit in LDS, rows padded by four
// entries so the sixteen rows a wavefront reads fall on different banks.
template <int CPIN, int COUT, int CPOUT, int EPI>
__global__ __launch_bounds__(256, 3) void k_conv(const uint16_t* __restrict__ in,
                                                 const uint16_t* __restrict__ wmat,
                                                 const float* __restrict__ bias,
                                                 const uint16_t* __restrict__ mask, void* out,
                                                 int n, const double* __restrict__ scal,
                                                 double* __restrict__ part) {
    constexpr int KC = (27 * CPIN + 15) / 16;
    constexpr int KW = KC * 16 + 4;              // LDS row of the weights (bf16 entries)
    constexpr int W8 = CPIN / 4;                 // 8-byte words per brick cell
    __shared__ __align__(16) uint64_t brick[kCBrick * W8];
    __shared__ __align__(16) uint16_t wl[16 * KW];
    const int tid = int(threadIdx.x);
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int col = lane & 15;                   // z within the segment; A row
    const int kq = lane >> 4;                    // which 4-wide k group
    for (int i = tid; i < 16 * KC * 4; i += 256) {
        const int row = i / (KC * 4), q = i - row * (KC * 4);
        *reinterpret_cast<uint64_t*>(&wl[row * KW + 4 * q]) =
            *(const WDM_GAS uint64_t*)(wmat + int64_t(row) * (KC * 16) + 4 * q);
    }
    auto a_op = [&](int ch) {
        bf16x4 a;
        const uint64_t w = *reinterpret_cast<const uint64_t*>(&wl[col * KW + ch * 16 + 4 * kq]);
        __builtin_memcpy(&a, &w, sizeof(a));
        return a;
    };
    const int tx = (n + kCTX - 1) / kCTX, ty = (n + kCTY - 1) / kCTY, tz = (n + kCTZ - 1) / kCTZ;
    const int64_t ntiles = int64_t(tx) * ty * tz;
    BrickRegs<W8> R;
    if (int64_t(blockIdx.x) < ntiles) brick_load<CPIN, W8>(R, in, blockIdx.x, n, tz, ty);
    double mass = 0.0;   // kEpiApply: this lane's cells, in tile order
    const float s_out = EPI == kEpiApply ? float(gldr(scal, 5)) : 0.0f;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int iz = int(t % tz);
        const int64_t r = t / tz;
        const int x0 = int(r / ty) * kCTX, y0 = int(r % ty) * kCTY, z0 = iz * kCTZ;
        brick_store<W8>(R, brick);
        __syncthreads();
        if (t + gridDim.x < ntiles) brick_load<CPIN, W8>(R, in, t + gridDim.x, n, tz, ty);
        // wavefront `wave` owns x = x0 + wave, y = y0 + s (s < 4), z = z0 + col
        f32x4 acc[kCTY];
#pragma unroll
        for (int s2 = 0; s2 < kCTY; ++s2) acc[s2] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (CPIN == 16) {
            // one K chunk per tap (16 channels).  For fixed (dx, dz) the four
            // segments and three dy offsets read only six brick rows (segment
            // s at offset dy is row s + dy): each B operand read from LDS
            // serves two MFMAs on average.
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                for (int dz = 0; dz < 3; ++dz) {
                    uint64_t braw[kCTY + 2];
#pragma unroll
                    for (int rr = 0; rr < kCTY + 2; ++rr)
                        braw[rr] = brick[(((wave + dx) * kCBY + rr) * kCBZ + col + dz) * W8 + kq];
#pragma unroll
                    for (int dy = 0; dy < 3; ++dy) {
                        const bf16x4 a = a_op(dx * 9 + dy * 3 + dz);
#pragma unroll
                        for (int s2 = 0; s2 < kCTY; ++s2) {
                            bf16x4 b;
                            __builtin_memcpy(&b, &braw[s2 + dy], sizeof(b));
                            acc[s2] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[s2], 0,
                                                                                0, 0);
                        }
                    }
                }
        } else {
#pragma unroll
            for (int ch = 0; ch < KC; ++ch) {
                const int k0 = ch * 16 + 4 * kq;
                const int tap = k0 / CPIN, c = k0 % CPIN;
                const bool live = k0 < 27 * CPIN;
                const int dx = tap / 9, dy = (tap / 3) % 3, dz = tap % 3;
                const int cell0 = ((wave + dx) * kCBY + dy) * kCBZ + col + dz;
                const bf16x4 a = a_op(ch);
#pragma unroll
                for (int s2 = 0; s2 < kCTY; ++s2) {
                    const uint64_t bw = live ? brick[(cell0 + s2 * kCBZ) * W8 + c / 4] : 0ull;
                    bf16x4 b;
                    __builtin_memcpy(&b, &bw, sizeof(b));
                    acc[s2] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[s2], 0, 0, 0);
                }
            }
        }
        // epilogue: lane holds out[cell][4*kq + q] of each segment
        const int x = x0 + wave, z = z0 + col, m0 = 4 * kq;
#pragma unroll
        for (int s2 = 0; s2 < kCTY; ++s2) {
            const int y = y0 + s2;
            if (x >= n || y >= n || z >= n) continue;
            const int64_t cell = (int64_t(x) * n + y) * n + z;
            if constexpr (EPI == kEpiBiasF32) {
                float* o = static_cast<float*>(out);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (m0 + q < COUT) gstr(o, cell * COUT + m0 + q, acc[s2][q] + gldr(bias, m0 + q));
            } else if constexpr (EPI == kEpiApply) {
                static_assert(COUT == 2, "the correction has two output channels");
                if (m0 != 0) continue;
                float* psi = static_cast<float*>(out);
                const float re = gldr(psi, 2 * cell) + s_out * (acc[s2][0] + gldr(bias, 0));
                const float im = gldr(psi, 2 * cell + 1) + s_out * (acc[s2][1] + gldr(bias, 1));
                gstr(psi, 2 * cell, re);
                gstr(psi, 2 * cell + 1, im);
                mass += double(re) * double(re) + double(im) * double(im);
            } else {
                if (m0 >= CPOUT) continue;
                uint16_t rq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float v = acc[s2][q];
                    if constexpr (EPI == kEpiBiasReluBf16) {
                        v = m0 + q < COUT ? fmaxf(v + gldr(bias, m0 + q), 0.0f) : 0.0f;
                    } else {
                        const float mk = bf2f(gldr(mask, cell * CPOUT + m0 + q));
                        v = (m0 + q < COUT && mk > 0.0f) ? v : 0.0f;
                    }
                    rq[q] = f2bf(v);
                }
                const uint64_t packed = uint64_t(rq[0]) | (uint64_t(rq[1]) << 16) |
                                        (uint64_t(rq[2]) << 32) | (uint64_t(rq[3]) << 48);
                gstr(reinterpret_cast<uint64_t*>(static_cast<uint16_t*>(out)),
                     (cell * CPOUT + m0) / 4, packed);
            }
        }
        __syncthreads();   // the next tile's brick overwrites this one
    }
    if constexpr (EPI == kEpiApply) {
        // the work-group's sum in a fixed order (lanes, then the four
        // wavefronts), reusing the brick's LDS
        double* red = reinterpret_cast<double*>(brick);
        red[tid] = mass;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        if (tid == 0) gstr(part, int64_t(blockIdx.x), red[0]);
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

// f32 [cells][cin] -> bf16 [cells][CP] (zero padded), channel c scaled by
// sc[sidx[c]] (the network's input scales, device doubles) when sc is given.
__global__ void k_pack_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t cells,
                            int cin, int cp, const double* __restrict__ sc) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= cells * cp) return;
    const int64_t p = i / cp;
    const int c = int(i % cp);
    float v = 0.0f;
    if (c < cin) {
        v = gldr(x, p * cin + c);
        if (sc) v *= float(gldr(sc, c < 2 ? 0 : 1));
    }
    gstr(y, i, f2bf(v));
}

// loss = sum (y - t)^2 / count in FP64 partials; dy = bf16(2 (y - t) / count)
// stored with CP channels.
// The target t is in the network's output units divided by s_out (read
// from *s_out when given): the network learns t / s_out.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             uint16_t* __restrict__ dy, double* __restrict__ part,
                                             int64_t cells, int cout, int cp,
                                             const double* __restrict__ s_out) {
    __shared__ double red[256];
    const int64_t count = cells * cout;
    const float inv = s_out ? float(1.0 / gldr(s_out, 0)) : 1.0f;
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < cells * cp;
         i += int64_t(gridDim.x) * 256) {
        const int64_t p = i / cp;
        const int c = int(i % cp);
        float g = 0.0f;
        if (c < cout) {
            const float d = gldr(y, p * cout + c) - gldr(t, p * cout + c) * inv;
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

// ---- the corrector applied to a member's state -------------------------------
// scal (device doubles): [1] mass before, [2] mass after, [3] s_psi, [4] s_phi,
// [5] s_out.  Reductions: a fixed grid of kMassBlocks work-groups, each
// summing a fixed range into its own FP64 partial (deterministic).
constexpr int kMassBlocks = 1024;

__device__ __forceinline__ double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

// Network inputs from the state, x0[p] = bf16(Re psi s_psi, Im psi s_psi,
// Phi s_phi, 0), and the FP64 partials of |psi|^2 (mass before the correction).
__global__ __launch_bounds__(256) void k_state_pack(const float* __restrict__ psi,
                                                    const float* __restrict__ phi,
                                                    uint16_t* __restrict__ x0, int64_t cells,
                                                    const double* __restrict__ scal,
                                                    double* __restrict__ part) {
    __shared__ double red[256];
    const float sp = float(gldr(scal, 3)), sf = float(gldr(scal, 4));
    double m = 0.0;
    for (int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x; p < cells;
         p += int64_t(gridDim.x) * 256) {
        const float re = gldr(psi, 2 * p), im = gldr(psi, 2 * p + 1);
        m += double(re) * double(re) + double(im) * double(im);
        const uint64_t packed = uint64_t(f2bf(re * sp)) | (uint64_t(f2bf(im * sp)) << 16) |
                                (uint64_t(f2bf(gldr(phi, p) * sf)) << 32);
        gstr(reinterpret_cast<uint64_t*>(x0), p, packed);
    }
    const double t = block_sum(m, red);
    if (threadIdx.x == 0) gstr(part, int64_t(blockIdx.x), t);
}

// out[slot] = sum of n partials in a fixed order (thread t adds t, t + 256,
// ..., then the work-group tree), one 256-thread work-group.
__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ part, int n,
                                                   double* __restrict__ out, int slot) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = int(threadIdx.x); i < n; i += 256) s += gldr(part, i);
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) gstr(out, slot, t);
}

// psi *= sqrt(mass before / mass after), the factor formed in FP64.
__global__ void k_rescale(float* __restrict__ psi, int64_t cells, const double* __restrict__ scal) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= 2 * cells) return;
    const double a = gldr(scal, 2);
    const float f = a > 0.0 ? float(sqrt(gldr(scal, 1) / a)) : 1.0f;
    gstr(psi, i, gldr(psi, i) * f);
}

// ---- training data --------------------------------------------------------
// A training pair from a member's state and a target field: x[p] = (Re psi,
// Im psi, Phi), y[p] = (Re, Im)(target - psi), both f32 channels last.
__global__ void k_pair(const float* __restrict__ psi, const float* __restrict__ phi,
                       const float* __restrict__ target, float* __restrict__ x,
                       float* __restrict__ y, int64_t cells) {
    const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (p >= cells) return;
    const float re = gldr(psi, 2 * p), im = gldr(psi, 2 * p + 1);
    gstr(x, 3 * p + 0, re);
    gstr(x, 3 * p + 1, im);
    gstr(x, 3 * p + 2, gldr(phi, p));
    gstr(y, 2 * p + 0, gldr(target, 2 * p) - re);
    gstr(y, 2 * p + 1, gldr(target, 2 * p + 1) - im);
}

// Moments of a training set, accumulated pair by pair into per-work-group
// FP64 rows (first pair: overwrite): [0] sum x0^2 + x1^2, [1] sum x2,
// [2] sum x2^2, [3] sum y0^2 + y1^2, [4] sum y0 + y1.
constexpr int kMoments = 5;
__global__ __launch_bounds__(256) void k_moments(const float* __restrict__ x,
                                                 const float* __restrict__ y, int64_t cells,
                                                 double* __restrict__ rows, int first) {
    __shared__ double red[256];
    double a[kMoments] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x; p < cells;
         p += int64_t(gridDim.x) * 256) {
        const double x0 = gldr(x, 3 * p), x1 = gldr(x, 3 * p + 1), x2 = gldr(x, 3 * p + 2);
        const double y0 = gldr(y, 2 * p), y1 = gldr(y, 2 * p + 1);
        a[0] += x0 * x0 + x1 * x1;
        a[1] += x2;
        a[2] += x2 * x2;
        a[3] += y0 * y0 + y1 * y1;
        a[4] += y0 + y1;
    }
    for (int f = 0; f < kMoments; ++f) {
        const double t = block_sum(a[f], red);
        if (threadIdx.x == 0) {
            double* r = rows + int64_t(blockIdx.x) * kMoments + f;
            gstr(r, 0, first ? t : gldr(r, 0) + t);
        }
        __syncthreads();
    }
}

// Scales from the moments of `count` cells (count = pairs x cells per pair):
// s_psi = 1 / rms|psi|, s_phi = 1 / std(Phi), s_out = std of the residual's
// components (population moments); written to scal[3..5].
__global__ __launch_bounds__(256) void k_fit_scales(const double* __restrict__ rows, double count,
                                                    double* __restrict__ scal) {
    __shared__ double red[256];
    double m[kMoments];
    for (int f = 0; f < kMoments; ++f) {
        double s = 0.0;
        for (int b = int(threadIdx.x); b < kMassBlocks; b += 256)
            s += gldr(rows, int64_t(b) * kMoments + f);
        m[f] = block_sum(s, red);
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double ms = m[0] / count;
    const double mean_phi = m[1] / count, var_phi = m[2] / count - mean_phi * mean_phi;
    const double mean_y = m[4] / (2.0 * count), var_y = m[3] / (2.0 * count) - mean_y * mean_y;
    gstr(scal, 3, ms > 0.0 ? 1.0 / sqrt(ms) : 1.0);
    gstr(scal, 4, var_phi > 0.0 ? 1.0 / sqrt(var_phi) : 1.0);
    gstr(scal, 5, var_y > 0.0 ? sqrt(var_y) : 1e-30);
}

__global__ void k_set_scales(double* __restrict__ scal, double s_psi, double s_phi, double s_out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    gstr(scal, 3, s_psi);
    gstr(scal, 4, s_phi);
    gstr(scal, 5, s_out);
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

// Persistent grid of the convolution: one work-group per tile up to `per_cu`
// per compute unit.  Eight at 4 input channels; three at 16, although their
// 34.8 KB of LDS and 72-76 VGPRs would allow four: at 128^3 the forward pass
// measured 155-158 us with three per CU, 170-176 us with four or with two.
static unsigned conv_blocks(int n, int per_cu) {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, c = 0;
        cus = (hipGetDevice(&dev) == hipSuccess &&
               hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
               c > 0) ? c : 256;
    }
    const int64_t tiles = int64_t((n + kCTX - 1) / kCTX) * ((n + kCTY - 1) / kCTY) *
                          ((n + kCTZ - 1) / kCTZ);
    const int64_t cap = int64_t(per_cu) * cus;
    return unsigned(tiles < cap ? tiles : cap);
}

hipError_t conv_forward_layer(hipStream_t s, int layer, const uint16_t* in, const uint16_t* w,
                              const float* b, void* out, int n) {
    if (layer == 0)
        k_conv<4, 16, 16, kEpiBiasReluBf16><<<conv_blocks(n, 8), 256, 0, s>>>(in, w, b, nullptr,
                                                                             out, n, nullptr, nullptr);
    else if (layer == 1)
        k_conv<16, 16, 16, kEpiBiasReluBf16><<<conv_blocks(n, 3), 256, 0, s>>>(in, w, b, nullptr,
                                                                              out, n, nullptr, nullptr);
    else
        k_conv<16, 2, 4, kEpiBiasF32><<<conv_blocks(n, 3), 256, 0, s>>>(in, w, b, nullptr, out, n,
                                                                        nullptr, nullptr);
    return hipGetLastError();
}

// Gradient wrt the input of layer `layer` (1 or 2), masked by that input's ReLU.
hipError_t conv_backward_data(hipStream_t s, int layer, const uint16_t* dz, const uint16_t* wbwd,
                              const uint16_t* act_in, uint16_t* dact, int n) {
    if (layer == 2)
        k_conv<4, 16, 16, kEpiMaskBf16><<<conv_blocks(n, 8), 256, 0, s>>>(dz, wbwd, nullptr,
                                                                         act_in, dact, n,
                                                                         nullptr, nullptr);
    else
        k_conv<16, 16, 16, kEpiMaskBf16><<<conv_blocks(n, 3), 256, 0, s>>>(dz, wbwd, nullptr,
                                                                          act_in, dact, n,
                                                                          nullptr, nullptr);
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
                          int cp, const double* scales) {
    k_pack_bf16<<<unsigned((cells * cp + 255) / 256), 256, 0, s>>>(x, y, cells, cin, cp, scales);
    return hipGetLastError();
}

hipError_t net_mse(hipStream_t s, const float* y, const float* t, uint16_t* dy, double* part,
                   double* out, int64_t cells, int cout, int cp, const double* s_out) {
    constexpr int kBlocks = 1024;
    k_mse<<<kBlocks, 256, 0, s>>>(y, t, dy, part, cells, cout, cp, s_out);
    k_sum_parts<<<1, 256, 0, s>>>(part, kBlocks, out, 0);
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

hipError_t net_state_pack(hipStream_t s, const float* psi, const float* phi, uint16_t* x0,
                          int64_t cells, double* scal, double* part) {
    k_state_pack<<<kMassBlocks, 256, 0, s>>>(psi, phi, x0, cells, scal, part);
    k_sum_parts<<<1, 256, 0, s>>>(part, kMassBlocks, scal, 1);
    return hipGetLastError();
}

// The network's last layer with the correction in its epilogue: psi +=
// s_out (layer output), the corrected mass summed per work-group and then in
// a fixed order into scal[2]; with `rescale`, psi *= sqrt(scal[1] / scal[2]).
hipError_t net_last_layer_apply(hipStream_t s, const uint16_t* in, const uint16_t* w,
                                const float* b, float* psi, int n, double* scal, double* part,
                                bool rescale) {
    const unsigned g = conv_blocks(n, 3);
    if (g > unsigned(kMassBlocks)) return hipErrorInvalidValue;   // the partials' capacity
    k_conv<16, 2, 4, kEpiApply><<<g, 256, 0, s>>>(in, w, b, nullptr, psi, n, scal, part);
    k_sum_parts<<<1, 256, 0, s>>>(part, int(g), scal, 2);
    const int64_t cells = int64_t(n) * n * n;
    if (rescale) k_rescale<<<unsigned((2 * cells + 255) / 256), 256, 0, s>>>(psi, cells, scal);
    return hipGetLastError();
}


hipError_t net_pair(hipStream_t s, const float* psi, const float* phi, const float* target,
                    float* x, float* y, int64_t cells) {
    k_pair<<<unsigned((cells + 255) / 256), 256, 0, s>>>(psi, phi, target, x, y, cells);
    return hipGetLastError();
}

hipError_t net_moments(hipStream_t s, const float* x, const float* y, int64_t cells, double* rows,
                       bool first) {
    k_moments<<<kMassBlocks, 256, 0, s>>>(x, y, cells, rows, first ? 1 : 0);
    return hipGetLastError();
}

hipError_t net_fit_scales(hipStream_t s, const double* rows, double count, double* scal) {
    k_fit_scales<<<1, 256, 0, s>>>(rows, count, scal);
    return hipGetLastError();
}

hipError_t net_set_scales(hipStream_t s, double* scal, double s_psi, double s_phi, double s_out) {
    k_set_scales<<<1, 64, 0, s>>>(scal, s_psi, s_phi, s_out);
    return hipGetLastError();
}

size_t net_moment_doubles() { return size_t(kMassBlocks) * kMoments; }

}  // namespace wdm
