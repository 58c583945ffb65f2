// Internal declarations shared by the HIP translation units of libwdm.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace wdm {

// Device accesses through pointers read out of the member table would compile
// to flat memory instructions (the compiler cannot prove they are global),
// which also hold the LDS wait counter.  These accessors cast to the global
// address space so loads, stores and atomics are global_* instructions.
#define WDM_GAS __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T gldr(const T* p, int64_t i) {
    return ((const WDM_GAS T*)p)[i];
}
template <typename T>
__device__ __forceinline__ void gstr(T* p, int64_t i, T v) {
    ((WDM_GAS T*)p)[i] = v;
}
__device__ __forceinline__ void gatomic_add(float* p, float v) {
    __builtin_amdgcn_global_atomic_fadd_f32((WDM_GAS float*)p, v);
}
__device__ __forceinline__ void gatomic_add(double* p, double v) {
    __builtin_amdgcn_global_atomic_fadd_f64((WDM_GAS double*)p, v);
}

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kTwoPi = 2.0 * kPi;

// Per-member device descriptor (one halo / box).  Lives in device memory so
// that a single launch can serve a whole size class of an ensemble.
struct MemberDev {
    // grids (C order [nx][ny][nz], z contiguous)
    void* psi;        // complex, n cells
    void* phi;        // real potential, n cells
    void* rho_b;      // real baryon density accumulator, n cells (zero between steps,
                      // except with static baryons, whose deposit it keeps)
    void* spec;       // complex half spectrum [nx][ny][nz/2] (kz = 0 .. nz/2-1)
    void* spec_nyq;   // complex Nyquist plane [nx][ny] (kz = nz/2)
    void* scratch;    // complex, n cells (diagnostics only)
    // kinetic factors of the call's dt, written once per wdm_step call and read by P3:
    // [0, nx) e_x(k_x); [nx, nx + ny nz) e_yz(k_y, k_z) / N at q = iy nz + iz.
    // 16 bytes per entry: (hi, lo) complex64 pair, or one complex128.
    void* kin;
    // absorbing-boundary factors of the step's dt, b_a = exp(-alpha dt g_a) at
    // the nodes: [0, nx) x, [nx, nx + ny) y, [nx + ny, nx + ny + nz) z (FP64)
    double* absorb;
    // vacuum boundary: zero-padded (2nx, 2ny, 2nz) complex work grid and the
    // real transform of the padded Green's function on it (null if periodic)
    void* pad;
    void* green;
    // external potential, real n cells, mean acceleration removed (null if none)
    void* ext;
    const void* tw_x;  // W_nx^m, m in [0, nx) (complex, plan precision)
    const void* tw_y;
    const void* tw_z;
    int32_t nx, ny, nz;
    int32_t substeps;        // particle leapfrog sub-steps per step (>= 1)
    int32_t static_baryons;  // 1: particles never move and rho_b is kept between steps
    int32_t deterministic;   // 1: particles deposit through the fixed-point grid rho_fx
    double lx, ly, lz;
    double eta;        // hbar / m
    double four_pi_G;
    double kappa;                  // local self-interaction (0 = none)
    double absorb_alpha, absorb_nb;  // absorbing boundary (alpha = 0: none)
    double inv_dx, inv_dy, inv_dz;   // n / L per axis
    double inv_lx, inv_ly, inv_lz;   // 1 / L per axis
    // time-step slots (device doubles): [0] dt in use, [1] dt_auto, [2] dt set by user,
    // [3] current time
    double* dt;
    // particles: structure of arrays, sorted by cell between re-sorts
    int64_t np;
    float *px, *py, *pz, *vx, *vy, *vz;
    int32_t* id;       // original index of each slot
    float *apx, *apy, *apz, *avx, *avy, *avz;  // sort staging
    int32_t* aid;
    uint32_t *key_a, *key_b, *idx_a, *idx_b, *hist;
    double particle_mass;
    // FP64 reduction staging
    double* partials;  // [kMaxPartials][kRedFields]
    double* results;   // [kRedFields]
    // stability watch, written by every P1 launch: [0, watch_n) the largest
    // |Phi|, [watch_n, 2 watch_n) the largest |psi|^2 (kicks with a
    // self-interaction only), as FP64 bit patterns compared as unsigned
    // integers (NaN above +inf), one slot per wavefront of the launch (no two
    // wavefronts share a slot); [2 watch_n, 2 watch_n + 2) the two maxima
    // folded by the check; all cleared by each check
    unsigned long long* watch;
    int64_t watch_n;
    // [0] largest |dt| / dt_max (Sec. 3.5) over the steps checked since
    // wdm_set_state, [1] 1 once a non-finite potential or density was seen
    double* stab;
    // deterministic deposit: 64-bit fixed-point accumulator grid (n cells;
    // null unless deterministic) holding round(value * fx_scale)
    unsigned long long* rho_fx;
    double fx_scale, fx_inv;
};

constexpr int kRedFields = 11;
constexpr int kRedBlocks = 1024;

// Launch context shared by all launchers.
struct Launch {
    hipStream_t stream;
    const MemberDev* members;   // device table
    int first;                  // first member index of the size class
    int count;                  // members in the class
};

enum KickMode : int { kHalfKick = 0, kFullKick = 1 };
enum ZOp : int { kZKickFft = 0, kZKickOnly = 1, kZPhiOnly = 2 };
// P5 operations: kDensInvFft inverse z-FFT of psi, density, R2C into the half
// spectrum; kDensDirect the same from psi in real space; kDensInvToPhi and
// kDensDirectToPhi stop at the density, written to Phi (the vacuum solve's
// input); kPhiR2C R2C of Phi into the half spectrum (its output).
enum DensOp : int {
    kDensInvFft = 0, kDensDirect = 1, kDensInvToPhi = 2, kDensDirectToPhi = 3, kPhiR2C = 4
};

// ---- FFT passes (passes_z.hip, passes_y.hip, passes_x.hip); `prec` is 0 for complex64, 1 for complex128 ----
bool axis_supported(int n);
// True where the axis length has a second FFT plan (the autotuner's choice).
bool axis_has_variant(int n);
// Whether a length has the wide-row plan (V = 2) of the strided passes.
bool axis_has_wide(int n);
bool axis_has_zcx(int n);   // z passes with a complex-exchange plan
// P1: half spectrum -> Phi (C2R along z), then kick and optionally z-FFT.
// `extended` selects the kick with the local self-interaction, the absorbing
// boundary and the external potential (needed when a member of the class has
// one; it runs the default FFT plan whatever `variant` says).
hipError_t launch_z_potential_kick(const Launch& L, int prec, int nx, int ny, int nz, ZOp op,
                                   KickMode kick, int variant = 0, bool extended = false);
// P2 / P4 on psi, P6 / P8 on the half spectrum (+ Nyquist plane).
hipError_t launch_y_fft_psi(const Launch& L, int prec, int nx, int ny, int nz, bool inverse,
                            int variant = 0);
hipError_t launch_y_fft_spec(const Launch& L, int prec, int nx, int ny, int nz, bool inverse,
                             int variant = 0);
// Kinetic factor tables e_x, e_yz / N of the dt in use (dt[0]) for every member
// of the class; max_entries = the largest nx + ny nz of the class.
hipError_t launch_kinetic_tables(const Launch& L, int prec, int64_t max_entries);
// P3: x forward, kinetic phase exp(-i eta |k|^2 dt/2)/N, x inverse.
hipError_t launch_x_kinetic(const Launch& L, int prec, int nx, int ny, int nz, int variant = 0);
// P5: z inverse of psi (optional), rho = |psi|^2 + rho_b (rho_b cleared except
// for the member of device index keep_member), R2C along z.  `rescale`
// (kDensDirect only): psi is first scaled by sqrt(rescale[1] / rescale[2]) and
// written back.
hipError_t launch_z_density(const Launch& L, int prec, int nx, int ny, int nz, DensOp op,
                            int variant = 0, int keep_member = -1,
                            const double* rescale = nullptr);
// P7: x forward, Green's function -4 pi G / |k|^2 / N, x inverse (+ Nyquist plane).
hipError_t launch_x_green(const Launch& L, int prec, int nx, int ny, int nz, int variant = 0);
// Plain 3D transforms between psi-shaped buffers: axis 0 = x, 1 = y, 2 = z.
// `which` selects the member field: 0 = psi, 1 = scratch.
hipError_t launch_axis_fft(const Launch& L, int prec, int nx, int ny, int nz, int axis,
                           bool inverse, int which);
// Transforms of the vacuum solve on the padded member table (nx, ny, nz the
// padded lengths): mode 0 density rows of Phi -> padded rows, forward z;
// 1 forward y (inputs y >= ny/2 zero); 2 inverse y (outputs y < ny/2 stored);
// 3 inverse z, real part of the first nz/2 values -> Phi.  Rows and pencils
// with x >= nx/2 are not touched.
hipError_t launch_vac_fft(const Launch& L, int prec, int nx, int ny, int nz, int mode);
// FP64 spectral kinetic-energy partials from scratch holding F_z F_y psi.
hipError_t launch_x_kinetic_energy(const Launch& L, int prec, int nx, int ny, int nz);

// ---- particles (particles.hip) ----
// mode 0: kick (tau) + drift (dt) + deposit; 1: kick only; 2: deposit only
// into rho_b; 3: deposit only into scratch (as real grid).  per_cu: resident
// work-groups per compute unit (0: the default, four).
hipError_t launch_particles(const Launch& L, int prec, int64_t max_np, int mode,
                            KickMode kick, bool det = false, int per_cu = 0);
// Stable radix sort by Morton cell key of every member of a size class.
hipError_t launch_particle_sort(const Launch& L, int64_t max_np, int nx, int ny, int nz);
hipError_t launch_particle_unsort(hipStream_t s, const MemberDev& m, float* pos_out,
                                  float* vel_out);
hipError_t launch_particle_upload(hipStream_t s, const MemberDev& m, const float* pos,
                                  const float* vel);

// ---- vacuum boundary and external potential (isolated.hip) ----
// Green's function on the padded grid (into pad), then its transform's real
// part into green (after the caller's forward transform of pad).
hipError_t launch_green_fill(const Launch& L, int prec, int64_t max_cells);
hipError_t launch_green_extract(const Launch& L, int prec, int64_t max_cells);
// x forward, times green, x inverse on the padded grid (L over the padded
// member table; nx, ny, nz the padded lengths).
hipError_t launch_x_mul_green(const Launch& L, int prec, int nx, int ny, int nz);
// Remove the mean acceleration of the member's ext (one member).
hipError_t launch_tidal_correct(const Launch& L, int prec, int64_t ncells);

// ---- diagnostics (diag.hip) ----
// Partials of K, Q, V, Px, Py, Pz, sum |psi|^2 (per 1/dV) into fields 0..6
// over `nblocks` work-groups; finish each with launch_reduce_finish.
hipError_t launch_diag_energies(const Launch& L, int prec, int nblocks);
// Mass-fraction radii (10%, ..., 90%) around the node `centre` into out[0..8]
// via a radial histogram hist[0..nbins) of squared node distances.
hipError_t launch_mass_radii(const Launch& L, int prec, int64_t ncells, const int centre[3],
                             double dx, double* hist, int64_t nbins, double* out);

// ---- reductions and small kernels (reduce.hip) ----
// fields of `results`: 0 mass, 1 e_kin, 2 sum rho Phi, 3 sum v^2, 4..6 sum v,
// 7 max |Phi|, 8 max |psi|^2, 9 sum |psi|^4, 10 sum rho Phi_ext
hipError_t launch_reduce_grid(const Launch& L, int prec, int64_t ncells, int what);
hipError_t launch_reduce_finish(const Launch& L, int field, int nblocks, bool is_max);
hipError_t launch_reduce_particles(const Launch& L, int64_t max_np);
hipError_t launch_dt_auto(const Launch& L, double zeta, double c_kin);
hipError_t launch_set_dt(const Launch& L, double dt, int mode);
// Absorbing-boundary factor tables of every member of the class from dt[0]
// (all ones where absorb_alpha is 0).
hipError_t launch_absorb_tables(const Launch& L);
hipError_t launch_advance_time(const Launch& L, int64_t nsteps);
// Slots of the stability watch per member: at least the wavefronts of any P1
// launch (one pencil or more per wavefront).
inline int64_t watch_slots(int nx, int ny) { return int64_t(nx) * ny + 1024; }
// 64-bit words of a member's watch: the two slot halves and their two totals.
inline int64_t watch_words(int nx, int ny) { return 2 * watch_slots(nx, ny) + 2; }
// Stability check after a wdm_step call: folds the watch slots (`slots` =
// watch_n of the class) into stab (|dt| / dt_max with dt_max = 0.5 min{c_kin
// dx^2 / eta, 2 pi eta / max|Phi|, 2 pi eta / (|kappa| max|psi|^2)}, Sec. 3.5)
// and clears them.
hipError_t launch_stability(const Launch& L, int64_t slots, double c_kin);
hipError_t launch_zero(hipStream_t s, void* p, size_t bytes);
hipError_t launch_copy_complex(hipStream_t s, void* dst, const void* src, int64_t n,
                               int dst_prec, int src_prec);
hipError_t launch_density_out(const Launch& L, int prec, int64_t ncells, void* out,
                              int include_baryons);
hipError_t launch_copy_real(hipStream_t s, void* dst, const void* src, int64_t n, int prec);
hipError_t launch_stream_copy(hipStream_t s, float4* dst, const float4* src, int64_t n);

}  // namespace wdm
