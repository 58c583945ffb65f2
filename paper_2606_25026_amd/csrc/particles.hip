// Baryon particles coupled to the wave through the mesh (Sec. 3.2.2, dynamic
// mode): the wave + baryon potential on the grid is differentiated by second
// order central differences (Sec. 3.1) and interpolated to the particles with
// cloud-in-cell weights; particles are kicked, drifted and deposited back onto
// the grid with the same weights.
//
// The deposit sorts nothing per step: particles are kept in Morton order of
// their cells (a stable LSD radix sort, re-run periodically), so the particles
// of a work-group fill a compact box of cells.  Each wavefront sums its
// contributions per run of equal cells; the runs are accumulated in an LDS box
// and each non-zero node costs one global atomic add per work-group.
#include "wdm_internal.hpp"

extern "C" __device__ __attribute__((const)) int __ockl_wfred_min_i32(int);
extern "C" __device__ __attribute__((const)) int __ockl_wfred_max_i32(int);

#include <algorithm>
#include <type_traits>

namespace wdm {

// i in [-n, 2n): periodic index without an integer division
__device__ __forceinline__ int wrapi(int i, int n) {
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

template <typename T>
struct CellW {
    int i, j, k;          // base cell (index in [0, n))
    T w[3][2];            // (1 - f, f) per axis
};

// s = x / dx, i = floor(s), f = s - i, formed in FP64 from the float position;
// the weights are kept in the grid precision T.
template <typename T>
__device__ __forceinline__ CellW<T> cic(float x, float y, float z, const MemberDev& m) {
    CellW<T> c;
    const double s[3] = {double(x) * m.inv_dx, double(y) * m.inv_dy, double(z) * m.inv_dz};
    const int n[3] = {m.nx, m.ny, m.nz};
    int ii[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double fl = floor(s[a]);
        const T f = T(s[a] - fl);
        ii[a] = wrapi(int(fl), n[a]);
        c.w[a][0] = T(1) - f;
        c.w[a][1] = f;
    }
    c.i = ii[0];
    c.j = ii[1];
    c.k = ii[2];
    return c;
}

// g = -grad Phi (central differences at the 8 CIC nodes), interpolated.
// P(a, b, d) returns Phi at cell (c.i - 1 + a, c.j - 1 + b, c.k - 1 + d),
// a, b, d in [0, 4); 32 of the 64 cells of that neighbourhood are read.
template <typename T, class F>
__device__ __forceinline__ void accel_from(const MemberDev& m, const CellW<T>& c, F&& P,
                                           float g[3]) {
    const T hx = T(0.5 * m.inv_dx), hy = T(0.5 * m.inv_dy), hz = T(0.5 * m.inv_dz);
    T gx = 0, gy = 0, gz = 0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                const T w = T(c.w[0][a]) * T(c.w[1][b]) * T(c.w[2][d]);
                // node (a+1, b+1, d+1) in the 4x4x4 neighbourhood
                gx += w * (P(a, b + 1, d + 1) - P(a + 2, b + 1, d + 1)) * hx;
                gy += w * (P(a + 1, b, d + 1) - P(a + 1, b + 2, d + 1)) * hy;
                gz += w * (P(a + 1, b + 1, d) - P(a + 1, b + 1, d + 2)) * hz;
            }
    g[0] = float(gx);
    g[1] = float(gy);
    g[2] = float(gz);
}

// 4- and 2-float rows at 4-byte alignment (global memory, address space 1).
typedef float wdm_row4 __attribute__((ext_vector_type(4), aligned(4)));
typedef float wdm_row2 __attribute__((ext_vector_type(2), aligned(4)));

template <typename T>
__device__ __forceinline__ void cic_accel(const T* __restrict__ phi, const MemberDev& m,
                                          const CellW<T>& c, float g[3]) {
    const int nx = m.nx, ny = m.ny, nz = m.nz;
    int ix[4], iy[4], iz[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        ix[d] = wrapi(c.i + d - 1, nx);
        iy[d] = wrapi(c.j + d - 1, ny);
        iz[d] = wrapi(c.k + d - 1, nz);
    }
    if constexpr (std::is_same<T, float>::value) {
        // The stencil's 32 values lie on 12 z-rows: 4 rows of 4 (a, b in
        // {1, 2}) and 8 rows of 2 (one of a, b in {0, 3}, d in {1, 2}).  Away
        // from the z faces each row is one vector load.
        if (c.k >= 1 && c.k + 2 < nz) {
            float v[4][4][4];
            // 32-bit row offsets (cells < 2^27 for axes <= 512): the loads
            // take the scalar base plus a 32-bit vector offset
            auto row = [&](int a, int b) {
                return phi + uint32_t((uint32_t(ix[a]) * uint32_t(ny) + uint32_t(iy[b])) *
                                      uint32_t(nz));
            };
#pragma unroll
            for (int a = 1; a < 3; ++a)
#pragma unroll
                for (int b = 1; b < 3; ++b) {
                    const wdm_row4 r =
                        *(const __attribute__((address_space(1))) wdm_row4*)(row(a, b) + c.k - 1);
                    v[a][b][0] = r.x;
                    v[a][b][1] = r.y;
                    v[a][b][2] = r.z;
                    v[a][b][3] = r.w;
                }
#pragma unroll
            for (int o = 0; o < 2; ++o)
#pragma unroll
                for (int u = 1; u < 3; ++u) {
                    const int e = o * 3;  // 0 or 3
                    const wdm_row2 rx =
                        *(const __attribute__((address_space(1))) wdm_row2*)(row(e, u) + c.k);
                    v[e][u][1] = rx.x;
                    v[e][u][2] = rx.y;
                    const wdm_row2 ry =
                        *(const __attribute__((address_space(1))) wdm_row2*)(row(u, e) + c.k);
                    v[u][e][1] = ry.x;
                    v[u][e][2] = ry.y;
                }
            accel_from(m, c, [&](int a, int b, int d) -> float { return v[a][b][d]; }, g);
            return;
        }
    }
    accel_from(m, c,
               [&](int a, int b, int d) -> T {
                   return gldr(phi, (int64_t(ix[a]) * ny + iy[b]) * nz + iz[d]);
               },
               g);
}

__device__ __forceinline__ float wrap_pos(double x, double L, double inv_l) {
    x -= L * floor(x * inv_l);
    float f = float(x);
    if (!(f >= 0.0f && f < float(L))) f = 0.0f;   // also a non-finite position
    return f;
}

// A deposit contribution in the accumulator type A: the grid precision T
// itself, or (deterministic deposit) the 64-bit fixed-point value
// round(v * scale), whose sums are exact and so independent of their order.
template <typename A, typename T>
__device__ __forceinline__ A to_acc(T v, double scale) {
    if constexpr (std::is_same<A, T>::value)
        return v;
    else
        return A(__double2ll_rn(double(v) * scale));
}

__device__ __forceinline__ void gatomic_add(unsigned long long* p, unsigned long long v) {
    atomicAdd(p, v);
}

// Per-run sums of the eight CIC contributions q * w of a wavefront: lanes
// holding the same base cell (consecutive after the cell sort) form a run; on
// return the run's first lane holds the run's sums in val[] and head = true.
// All 64 lanes of the wavefront must call this together.
template <typename T, typename A>
__device__ __forceinline__ bool wave_runs(const MemberDev& m, const CellW<T>& c, T q, bool act,
                                          A val[8], double scale) {
    const int lane = int(__lane_id());
    const int64_t key = act ? (int64_t(c.i) * m.ny + c.j) * m.nz + c.k : -1 - lane;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int d = 0; d < 2; ++d)
                val[a * 4 + b * 2 + d] =
                    act ? to_acc<A>(T(q * c.w[0][a] * c.w[1][b] * c.w[2][d]), scale) : A(0);
    // run heads: lanes whose key differs from the previous lane's
    const int64_t prev = __shfl_up(key, 1);
    const bool head = lane == 0 || prev != key;
    const unsigned long long heads = __ballot(head);
    const unsigned long long upto = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    const int seg = __popcll(heads & upto);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int oseg = __shfl_down(seg, off);
        const bool take = (lane + off < 64) && (oseg == seg);
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const A o = __shfl_down(val[v], off);
            if (take) val[v] += o;
        }
    }
    return head && act;
}

// Deposit q * w into `grid` at the 8 nodes of cell c, one global atomic add
// per node and wavefront run.
template <typename T, typename A>
__device__ __forceinline__ void deposit_wave(A* __restrict__ grid, const MemberDev& m,
                                             const CellW<T>& c, T q, bool act, double scale) {
    A val[8];
    if (!wave_runs(m, c, q, act, val, scale)) return;
    const int nx = m.nx, ny = m.ny, nz = m.nz;
    const int i1 = c.i + 1 == nx ? 0 : c.i + 1;
    const int j1 = c.j + 1 == ny ? 0 : c.j + 1;
    const int k1 = c.k + 1 == nz ? 0 : c.k + 1;
    const int I[2] = {c.i, i1}, J[2] = {c.j, j1}, K[2] = {c.k, k1};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int d = 0; d < 2; ++d)
                gatomic_add(&grid[(int64_t(I[a]) * ny + J[b]) * nz + K[d]],
                            A(val[a * 4 + b * 2 + d]));
}

// LDS staging of a work-group's deposit: 16 KB of nodes.
template <typename T>
constexpr int tile_nodes() {
    return 16384 / int(sizeof(T));
}
constexpr int kParticleWG = 256;

// wavefront minimum / maximum (DPP reductions)
__device__ __forceinline__ int wave_min(int v) { return __ockl_wfred_min_i32(v); }
__device__ __forceinline__ int wave_max(int v) { return __ockl_wfred_max_i32(v); }

// Work-group deposit.  The particles of a work-group are consecutive in
// Morton order, so their cells usually fill a small box: if that box (plus the
// upper CIC node) holds at most tile_nodes<T>() nodes, the group accumulates
// into LDS and issues one global atomic add per non-zero node; otherwise each
// wavefront deposits its runs directly.  Every lane of the work-group must
// call this (inactive lanes pass act = false).
template <typename T, typename A>
__device__ __forceinline__ void deposit_group(A* __restrict__ grid, const MemberDev& m,
                                              const CellW<T>& c, T q, bool act, double scale) {
    __shared__ A tile[tile_nodes<A>()];
    __shared__ int box[6];
    const int tid = int(threadIdx.x);
    constexpr int kBig = 1 << 30;
    const int lo0 = wave_min(act ? c.i : kBig), lo1 = wave_min(act ? c.j : kBig),
              lo2 = wave_min(act ? c.k : kBig);
    const int hi0 = wave_max(act ? c.i : -1), hi1 = wave_max(act ? c.j : -1),
              hi2 = wave_max(act ? c.k : -1);
    if (tid == 0) {
        box[0] = box[1] = box[2] = kBig;
        box[3] = box[4] = box[5] = -1;
    }
    __syncthreads();
    if (__lane_id() == 0) {
        atomicMin(&box[0], lo0);
        atomicMin(&box[1], lo1);
        atomicMin(&box[2], lo2);
        atomicMax(&box[3], hi0);
        atomicMax(&box[4], hi1);
        atomicMax(&box[5], hi2);
    }
    __syncthreads();
    if (box[3] < 0) return;  // no particle in the work-group (uniform)
    const int i0 = box[0], j0 = box[1], k0 = box[2];
    const int ex = box[3] - i0 + 2, ey = box[4] - j0 + 2, ez = box[5] - k0 + 2;
    // extents are at most n + 1 <= 513 each, so the product fits in int64
    const int64_t vol64 = int64_t(ex) * ey * ez;
    if (vol64 > tile_nodes<A>()) {
        deposit_wave(grid, m, c, q, act, scale);
        return;
    }
    const int vol = int(vol64);
    for (int t = tid; t < vol; t += kParticleWG) tile[t] = A(0);
    __syncthreads();
    A val[8];
    if (wave_runs(m, c, q, act, val, scale)) {
        const int base = ((c.i - i0) * ey + (c.j - j0)) * ez + (c.k - k0);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int d = 0; d < 2; ++d)
                    atomicAdd(&tile[base + (a * ey + b) * ez + d], val[a * 4 + b * 2 + d]);
    }
    __syncthreads();
    const int nx = m.nx, ny = m.ny, nz = m.nz;
    const int eyz = ey * ez;
    // (ti, tj, tk) of node t = tid, advanced by the stride kParticleWG with
    // carries: two divisions per chunk instead of two per node
    int ti = tid / eyz, tj = (tid - ti * eyz) / ez, tk = tid - ti * eyz - tj * ez;
    const int si = kParticleWG / eyz, sj = (kParticleWG - si * eyz) / ez,
              sk = kParticleWG - si * eyz - sj * ez;
    for (int t = tid; t < vol; t += kParticleWG) {
        const A v = tile[t];
        const int ci = ti, cj = tj, ck = tk;
        tk += sk;
        tj += sj;
        ti += si;
        if (tk >= ez) {
            tk -= ez;
            ++tj;
        }
        if (tj >= ey) {
            tj -= ey;
            ++ti;
        }
        if (v == A(0)) continue;
        // i0 + ci <= max cell + 1 <= n: one wrap at most
        int gi = i0 + ci, gj = j0 + cj, gk = k0 + ck;
        if (gi >= nx) gi -= nx;
        if (gj >= ny) gj -= ny;
        if (gk >= nz) gk -= nz;
        gatomic_add(&grid[(int64_t(gi) * ny + gj) * nz + gk], v);
    }
}

// mode 0: kick + drift + deposit into rho_b; 1: kick only; 2: deposit into
// rho_b; 3: deposit into scratch (as a real grid).
//
// Persistent work-groups: at most `per_cu` per compute unit are launched and
// each walks the member's 256-particle chunks with a grid stride.  Beside
// longer y/x/y passes (the 256^3 step) four per CU leave them most of the
// machine (0.4065 against 0.4103 ms per step with eight); where the particles
// are the step's longer branch (10^6 particles on 128^3) eight per CU shorten
// it (0.1146 against 0.1176 ms), and alone the kernel runs 44.5 against
// 47 us at 256^3 + 10^6.
constexpr int kGroupsPerCU = 4;

// With S = m.substeps leapfrog sub-steps of h = dt / S (Sec. 3.2.2), mode 0
// runs the opening (or merged) kick, then S drifts with a full kick of h in
// the same potential between them; the closing half kick of h/2 is mode 1
// after the step's Poisson solve.  Static baryons skip modes 0 and 1.
template <typename T, bool DET>
__global__ __launch_bounds__(kParticleWG) void k_particles(const MemberDev* __restrict__ mems,
                                                           int first, int mode, int kick) {
    const MemberDev& m = mems[first + blockIdx.y];
    if (mode <= 1 && m.static_baryons) return;   // uniform over the work-group
    const double dt = gldr(m.dt, 0);
    const int S = m.substeps;
    const double h = dt / S;
    for (int64_t grp = blockIdx.x; grp * kParticleWG < m.np; grp += gridDim.x) {
        const int64_t i = grp * kParticleWG + threadIdx.x;
        const bool act = i < m.np;
        const int64_t ii = act ? i : 0;
        float x = gldr(m.px, ii), y = gldr(m.py, ii), z = gldr(m.pz, ii);
        if (mode <= 1) {
            float vx = gldr(m.vx, ii), vy = gldr(m.vy, ii), vz = gldr(m.vz, ii);
            float tau = float(kick == kFullKick ? h : 0.5 * h);
            for (int sub = 0;; ++sub) {
                const CellW<T> c = cic<T>(x, y, z, m);
                float g[3];
                cic_accel(static_cast<const T*>(m.phi), m, c, g);
                vx += g[0] * tau;
                vy += g[1] * tau;
                vz += g[2] * tau;
                if (mode == 1) break;
                x = wrap_pos(double(x) + double(vx) * h, m.lx, m.inv_lx);
                y = wrap_pos(double(y) + double(vy) * h, m.ly, m.inv_ly);
                z = wrap_pos(double(z) + double(vz) * h, m.lz, m.inv_lz);
                if (sub + 1 == S) break;
                tau = float(h);   // the two half kicks between sub-steps
            }
            if (mode == 0) {
                if (act) {
                    gstr(m.px, i, x);
                    gstr(m.py, i, y);
                    gstr(m.pz, i, z);
                }
            }
            if (act) {
                gstr(m.vx, i, vx);
                gstr(m.vy, i, vy);
                gstr(m.vz, i, vz);
            }
            if (mode == 1) continue;  // uniform; no barrier in this mode
        }
        const T q = T(m.particle_mass * m.inv_dx * m.inv_dy * m.inv_dz);
        const CellW<T> c = cic<T>(x, y, z, m);
        if constexpr (DET) {
            // fixed-point sums, turned into the real grid by k_fixed_to_real
            deposit_group(m.rho_fx, m, c, q, act, m.fx_scale);
        } else {
            T* grid = static_cast<T*>(mode == 3 ? m.scratch : m.rho_b);
            deposit_group(grid, m, c, q, act, 0.0);
        }
        __syncthreads();  // the next chunk reuses the group's LDS box and tile
    }
}

// Compute units of the current device (queried once).
static int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            n > 0)
            cus = n;
        else
            cus = 256;
    }
    return cus;
}

// Deterministic deposit, second half: the fixed-point grid of each member of
// the class becomes the real grid (rho_b, or scratch for `to_scratch`) and is
// cleared.  With skip_static, members with static baryons keep their rho_b
// (the step deposits nothing for them).
template <typename T>
__global__ __launch_bounds__(256) void k_fixed_to_real(const MemberDev* __restrict__ mems,
                                                       int first, int to_scratch, int skip_static) {
    const MemberDev& m = mems[first + blockIdx.y];
    if (skip_static && m.static_baryons) return;
    if (m.rho_fx == nullptr) return;
    T* dst = static_cast<T*>(to_scratch ? m.scratch : m.rho_b);
    const int64_t n = int64_t(m.nx) * m.ny * m.nz;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        const unsigned long long v = gldr(m.rho_fx, i);
        gstr(dst, i, T(double((long long)v) * m.fx_inv));
        gstr(m.rho_fx, i, 0ull);
    }
}

hipError_t launch_particles(const Launch& L, int prec, int64_t max_np, int mode,
                            KickMode kick, bool det, int per_cu) {
    if (max_np <= 0) return hipSuccess;
    if (per_cu <= 0) per_cu = kGroupsPerCU;
    const int64_t chunks = (max_np + kParticleWG - 1) / kParticleWG;
    const int64_t cap = int64_t(per_cu) * device_cus();
    dim3 grid(unsigned(chunks < cap ? chunks : cap), unsigned(L.count));
    const bool fx = det && mode != 1;   // mode 1 deposits nothing
    if (prec) {
        if (fx)
            k_particles<double, true><<<grid, kParticleWG, 0, L.stream>>>(L.members, L.first,
                                                                          mode, int(kick));
        else
            k_particles<double, false><<<grid, kParticleWG, 0, L.stream>>>(L.members, L.first,
                                                                           mode, int(kick));
    } else {
        if (fx)
            k_particles<float, true><<<grid, kParticleWG, 0, L.stream>>>(L.members, L.first,
                                                                         mode, int(kick));
        else
            k_particles<float, false><<<grid, kParticleWG, 0, L.stream>>>(L.members, L.first,
                                                                          mode, int(kick));
    }
    if (!fx) return hipGetLastError();
    if (const hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    const dim3 cg(unsigned(4 * device_cus()), unsigned(L.count));
    const int to_scratch = mode == 3 ? 1 : 0, skip_static = mode == 0 ? 1 : 0;
    if (prec)
        k_fixed_to_real<double><<<cg, 256, 0, L.stream>>>(L.members, L.first, to_scratch,
                                                          skip_static);
    else
        k_fixed_to_real<float><<<cg, 256, 0, L.stream>>>(L.members, L.first, to_scratch,
                                                         skip_static);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// upload / download (AoS [Np][3] <-> SoA, original order via id)
// ---------------------------------------------------------------------------
__global__ void k_upload(MemberDev m, const float* __restrict__ pos, const float* __restrict__ vel) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= m.np) return;
    m.px[i] = wrap_pos(double(pos[3 * i + 0]), m.lx, m.inv_lx);
    m.py[i] = wrap_pos(double(pos[3 * i + 1]), m.ly, m.inv_ly);
    m.pz[i] = wrap_pos(double(pos[3 * i + 2]), m.lz, m.inv_lz);
    m.vx[i] = vel[3 * i + 0];
    m.vy[i] = vel[3 * i + 1];
    m.vz[i] = vel[3 * i + 2];
    m.id[i] = int32_t(i);
}

__global__ void k_unsort(MemberDev m, float* __restrict__ pos, float* __restrict__ vel) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= m.np) return;
    const int64_t o = m.id[i];
    if (pos) {
        pos[3 * o + 0] = m.px[i];
        pos[3 * o + 1] = m.py[i];
        pos[3 * o + 2] = m.pz[i];
    }
    if (vel) {
        vel[3 * o + 0] = m.vx[i];
        vel[3 * o + 1] = m.vy[i];
        vel[3 * o + 2] = m.vz[i];
    }
}

hipError_t launch_particle_upload(hipStream_t s, const MemberDev& m, const float* pos,
                                  const float* vel) {
    if (m.np <= 0) return hipSuccess;
    k_upload<<<unsigned((m.np + 255) / 256), 256, 0, s>>>(m, pos, vel);
    return hipGetLastError();
}

hipError_t launch_particle_unsort(hipStream_t s, const MemberDev& m, float* pos, float* vel) {
    if (m.np <= 0) return hipSuccess;
    k_unsort<<<unsigned((m.np + 255) / 256), 256, 0, s>>>(m, pos, vel);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of the particles by cell index (8-bit digits)
// ---------------------------------------------------------------------------
constexpr int kSortTile = 4096;   // keys per block: 256 lanes x 16 rounds

// Spread the low 10 bits of v to every third bit.
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Sort kernels work on a size class of members at once: blockIdx.y selects
// the member in the device table, each member sorts its own np particles with
// its own histogram (members of a class share the key width), and work-groups
// beyond a member's range return at once.  Members with at most one particle
// skip every stage.
__device__ __forceinline__ int sort_tiles(int64_t np) {
    return int((np + kSortTile - 1) / kSortTile);
}

// Sort key: Morton (bit-interleaved) index of the particle's cell, so that
// particles close in space are close in memory in all three directions and a
// work-group's force gathers and deposits stay within a compact patch.
__global__ void k_make_keys(const MemberDev* __restrict__ mems, int first) {
    const MemberDev& m = mems[first + blockIdx.y];
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= m.np) return;
    const CellW<float> c = cic<float>(m.px[i], m.py[i], m.pz[i], m);
    m.key_a[i] = (spread3(uint32_t(c.i)) << 2) | (spread3(uint32_t(c.j)) << 1) |
                 spread3(uint32_t(c.k));
    m.idx_a[i] = uint32_t(i);
}

// Lanes of the wavefront holding the same 8-bit digit (among `valid` lanes).
__device__ __forceinline__ unsigned long long match_digit(uint32_t d, bool valid) {
    unsigned long long mask = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
        const bool on = (d >> bit) & 1u;
        const unsigned long long bb = __ballot(on);
        mask &= on ? bb : ~bb;
    }
    return mask;
}

// Per-block digit counts of pass `pass` (keys in key_a for even passes, key_b
// for odd).  Keys of one block mostly share their high digits (particles are
// clustered), so equal digits are first counted across the wavefront and one
// lane per digit adds the group size.
__global__ __launch_bounds__(256) void k_radix_hist(const MemberDev* __restrict__ mems, int first,
                                                    int pass) {
    const MemberDev& m = mems[first + blockIdx.y];
    const int nb = sort_tiles(m.np);
    if (m.np <= 1 || int(blockIdx.x) >= nb) return;  // uniform per block
    const uint32_t* keys = (pass & 1) ? m.key_b : m.key_a;
    const int shift = 8 * pass;
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int lane = int(threadIdx.x) & 63;
    const unsigned long long lt = (1ull << lane) - 1ull;
    const int64_t b0 = int64_t(blockIdx.x) * kSortTile;
    for (int r = 0; r < kSortTile / 256; ++r) {
        const int64_t i = b0 + r * 256 + threadIdx.x;
        const bool valid = i < m.np;
        const uint32_t d = valid ? (keys[i] >> shift) & 255u : 0u;
        const unsigned long long mask = match_digit(d, valid);
        if (valid && __popcll(mask & lt) == 0) atomicAdd(&cnt[d], uint32_t(__popcll(mask)));
    }
    __syncthreads();
    m.hist[int64_t(threadIdx.x) * nb + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of the digit-major histogram hist[d * nb + b] in two small
// kernels: each of 256 blocks scans one digit's column over the nb tile blocks
// (and records the digit total after the histogram, at hist + 256 nb); one
// block then scans the 256 totals, which k_radix_scatter adds as the digit
// base.
__global__ __launch_bounds__(256) void k_scan_digit(const MemberDev* __restrict__ mems,
                                                    int first) {
    const MemberDev& m = mems[first + blockIdx.y];
    if (m.np <= 1) return;
    const int nb = sort_tiles(m.np);
    __shared__ uint32_t s[256];
    uint32_t* col = m.hist + int64_t(blockIdx.x) * nb;
    uint32_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 256) {
        const int b = b0 + int(threadIdx.x);
        const uint32_t v = b < nb ? col[b] : 0u;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const uint32_t t = int(threadIdx.x) >= off ? s[threadIdx.x - off] : 0u;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (b < nb) col[b] = carry + s[threadIdx.x] - v;
        carry += s[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) m.hist[int64_t(256) * nb + blockIdx.x] = carry;
}

__global__ __launch_bounds__(256) void k_scan_totals(const MemberDev* __restrict__ mems,
                                                     int first) {
    const MemberDev& m = mems[first + blockIdx.y];
    if (m.np <= 1) return;
    uint32_t* totals = m.hist + int64_t(256) * sort_tiles(m.np);
    __shared__ uint32_t s[256];
    const uint32_t v = totals[threadIdx.x];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t t = int(threadIdx.x) >= off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    totals[threadIdx.x] = s[threadIdx.x] - v;
}

// Stable scatter of pass `pass`: (key_a, idx_a) -> (key_b, idx_b) for even
// passes, the reverse for odd ones.
__global__ __launch_bounds__(256) void k_radix_scatter(const MemberDev* __restrict__ mems,
                                                       int first, int pass) {
    const MemberDev& m = mems[first + blockIdx.y];
    const int nb = sort_tiles(m.np);
    if (m.np <= 1 || int(blockIdx.x) >= nb) return;  // uniform per block
    const bool odd = (pass & 1) != 0;
    const uint32_t* kin = odd ? m.key_b : m.key_a;
    const uint32_t* vin = odd ? m.idx_b : m.idx_a;
    uint32_t* kout = odd ? m.key_a : m.key_b;
    uint32_t* vout = odd ? m.idx_a : m.idx_b;
    const int shift = 8 * pass;
    const uint32_t* hist = m.hist;
    const uint32_t* totals = m.hist + int64_t(256) * nb;
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[4][256];
    const int tid = int(threadIdx.x), lane = tid & 63, wave = tid >> 6;
    base[tid] = totals[tid] + hist[int64_t(tid) * nb + blockIdx.x];
    for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const unsigned long long lt = (1ull << lane) - 1ull;
    const int64_t b0 = int64_t(blockIdx.x) * kSortTile;
    for (int r = 0; r < kSortTile / 256; ++r) {
        const int64_t i = b0 + r * 256 + tid;
        const bool valid = i < m.np;
        const uint32_t k = valid ? kin[i] : 0u;
        const uint32_t d = (k >> shift) & 255u;
        const unsigned long long mask = match_digit(d, valid);
        const int rank = __popcll(mask & lt);
        if (valid && rank == 0) wcnt[wave][d] = uint32_t(__popcll(mask));
        __syncthreads();
        if (valid) {
            uint32_t off = base[d] + uint32_t(rank);
            for (int w = 0; w < wave; ++w) off += wcnt[w][d];
            kout[off] = k;
            vout[off] = vin[i];
        }
        __syncthreads();
        base[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
        for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
        __syncthreads();
    }
}

// Particles into sorted order through the staging arrays; the permutation
// is in idx_a after an even number of passes, idx_b after an odd number.
__global__ void k_gather_sorted(const MemberDev* __restrict__ mems, int first, int passes) {
    const MemberDev& m = mems[first + blockIdx.y];
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (m.np <= 1 || i >= m.np) return;  // one particle or none: nothing to reorder
    const uint32_t s = ((passes & 1) ? m.idx_b : m.idx_a)[i];
    m.apx[i] = m.px[s];
    m.apy[i] = m.py[s];
    m.apz[i] = m.pz[s];
    m.avx[i] = m.vx[s];
    m.avy[i] = m.vy[s];
    m.avz[i] = m.vz[s];
    m.aid[i] = m.id[s];
}

__global__ void k_copy_back(const MemberDev* __restrict__ mems, int first) {
    const MemberDev& m = mems[first + blockIdx.y];
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (m.np <= 1 || i >= m.np) return;
    m.px[i] = m.apx[i];
    m.py[i] = m.apy[i];
    m.pz[i] = m.apz[i];
    m.vx[i] = m.avx[i];
    m.vy[i] = m.avy[i];
    m.vz[i] = m.avz[i];
    m.id[i] = m.aid[i];
}

int sort_blocks(int64_t np) { return int((np + kSortTile - 1) / kSortTile); }

hipError_t launch_particle_sort(const Launch& L, int64_t max_np, int nx, int ny, int nz) {
    if (max_np <= 1) return hipSuccess;
    const unsigned y = unsigned(L.count);
    const dim3 g(unsigned((max_np + 255) / 256), y);
    const dim3 t(unsigned(sort_blocks(max_np)), y);
    int axis_bits = 0;
    while ((1 << axis_bits) < std::max(nx, std::max(ny, nz))) ++axis_bits;
    const int passes = (3 * axis_bits + 7) / 8;   // 8-bit digits of the Morton key
    k_make_keys<<<g, 256, 0, L.stream>>>(L.members, L.first);
    for (int pass = 0; pass < passes; ++pass) {
        k_radix_hist<<<t, 256, 0, L.stream>>>(L.members, L.first, pass);
        k_scan_digit<<<dim3(256, y), 256, 0, L.stream>>>(L.members, L.first);
        k_scan_totals<<<dim3(1, y), 256, 0, L.stream>>>(L.members, L.first);
        k_radix_scatter<<<t, 256, 0, L.stream>>>(L.members, L.first, pass);
    }
    k_gather_sorted<<<g, 256, 0, L.stream>>>(L.members, L.first, passes);
    k_copy_back<<<g, 256, 0, L.stream>>>(L.members, L.first);
    return hipGetLastError();
}

}  // namespace wdm
