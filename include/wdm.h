/*
 * wdm.h -- C ABI of the MI355X split-step Schroedinger-Poisson library.
 *
 * The library advances a wave-dark-matter field psi coupled to N-body baryon
 * particles with the kick-drift-kick split-step Fourier method of Meng & Dong,
 * "WaveDM.jl" (Sec. 3.1, Eq. SPE_solver_KDK and Algorithm 1), in code units
 * (Sec. 2.2, Eq. SPE_dimensionless) on a periodic box:
 *
 *     i d(psi)/dt = -(eta/2) lap(psi) + (1/eta) Phi psi,     eta = hbar/m
 *     lap(Phi)    = 4 pi G (|psi|^2 + rho_b - mean),
 *
 * with the periodic FFT Poisson solver of Sec. 3.2.1 and the dynamic baryon
 * mode of Sec. 3.2.2 (particles feed rho_b through a cloud-in-cell deposit and
 * feel -grad Phi, central differences of Sec. 3.1, CIC-interpolated).
 * Optional, per member (wdm_config): a local self-interaction kappa |psi|^2
 * and an absorbing boundary (Sec. 2.2, 3.1), static baryons and particle
 * sub-steps (Sec. 3.2.2), the vacuum gravity boundary (Sec. 3.2.1) and an
 * external tidal potential (Sec. 4.3); wdm_diagnostics gives the paper's halo
 * diagnostics (Sec. 3.6, App. A.1).
 *
 * Conventions shared by every entry point:
 *  - Grids are C-ordered [nx][ny][nz] with z contiguous; node i sits at
 *    x_i = i * lx / nx (periodic reading of the grid of Sec. 3.1).
 *  - psi buffers are interleaved complex: complex64 (float re, im) when the
 *    plan precision is WDM_C64, complex128 for WDM_C128.  Real grids (density,
 *    potential) are float for WDM_C64 and double for WDM_C128.
 *  - Particle buffers are float32 [n_particles][3], positions in [0, L).
 *  - All pointers named "dev" are device pointers owned by the caller; the
 *    library reads them during the call (stream-ordered on the plan's stream)
 *    and keeps no reference to them afterwards.  Host pointers are noted.
 *  - All device memory the plan needs lives in one caller-provided workspace
 *    (wdm_workspace_bytes); the library never allocates device memory.
 *  - Every call is ordered on the plan's HIP stream.  Only wdm_plan_create,
 *    wdm_energy, wdm_diagnostics, wdm_autotune, wdm_profile_read and
 *    wdm_copy_bandwidth synchronise with the host.
 *  - On an error nothing is launched, the plan keeps its state and
 *    wdm_last_error() describes the failure (thread-local string).
 *  - A plan is not thread safe; distinct plans are independent.
 */
#ifndef WDM_H
#define WDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wdm_plan wdm_plan;

typedef enum {
    WDM_OK = 0,
    WDM_EINVAL = 1,       /* bad argument (shape, size, index, null pointer) */
    WDM_ENOMEM = 2,       /* workspace too small */
    WDM_EDEVICE = 3,      /* a HIP call failed */
    WDM_ESTATE = 4,       /* call not valid in the plan's state (e.g. step before set_state) */
    WDM_EUNSTABLE = 5,    /* non-finite state or CFL violation detected */
    WDM_EUNSUPPORTED = 6  /* axis length or option not built */
} wdm_status;

typedef enum { WDM_C64 = 0, WDM_C128 = 1 } wdm_precision;

enum { WDM_BARYON_DYNAMIC = 0, WDM_BARYON_STATIC = 1 };

/* Bits of wdm_config.flags.
 *
 * WDM_DETERMINISTIC_DEPOSIT (must be the same on every member of a plan):
 * results are bitwise reproducible -- from run to run, between graph replays
 * and direct launches, and across a state saved between wdm_step calls
 * (wdm_get_psi, wdm_particles, wdm_energy's t) and set again with
 * wdm_set_state, on this plan or another with the same members.  The CIC
 * deposit (Sec. 3.2.2) sums 64-bit fixed-point contributions round(q w 2^S)
 * (S per member, such that all the member's particle mass on one node stays
 * below 2^62), so its sums are exact whatever the order of the particles or of
 * the atomic additions; and every wdm_step call starts by rebuilding the
 * potential from the synchronised state (one Poisson solve per call), exactly
 * as wdm_set_state builds it.  Costs an n-cell 8-byte grid per member and a
 * conversion pass per step.
 *
 * WDM_STRICT_CFL: a step above the CFL bound of Sec. 3.5 makes the next
 * wdm_energy / wdm_diagnostics call fail with WDM_EUNSTABLE (without it the
 * bound is only reported, wdm_energy_t.cfl_ratio).  Every step checks, on the
 * device, |dt| <= dt_max = 0.5 min{(4 / (3 pi)) dx_min^2 / eta,
 * 2 pi eta / max|Phi|, 2 pi eta / (|kappa| max|psi|^2)} with the maxima of the
 * potentials its kicks used; a non-finite potential or density always makes
 * those calls fail with WDM_EUNSTABLE.  The check stays set until
 * wdm_set_state.
 *
 * The kick and drift phase arguments are always formed in FP64 and reduced
 * mod 2 pi (there is no FP32-argument mode). */
#define WDM_DETERMINISTIC_DEPOSIT 0x1u
#define WDM_STRICT_CFL 0x2u
enum { WDM_BOUNDARY_PERIODIC = 0, WDM_BOUNDARY_VACUUM = 1 };

/* One box (an ensemble has several). */
typedef struct {
    int32_t nx, ny, nz;        /* each in {16,32,64,96,128,192,256,384,512} */
    double lx, ly, lz;         /* box lengths; dx = lx / nx */
    double hbar_over_m;        /* eta (1 in code units, Sec. 2.2) */
    double four_pi_G;          /* Poisson prefactor (Sec. 3.2.1); 0 = free equation */
    int64_t n_particles;       /* baryon particles (0 = none) */
    double particle_mass;      /* equal-mass particles */
    int32_t precision;         /* wdm_precision; all members of a plan share it */
    uint32_t flags;            /* WDM_DETERMINISTIC_DEPOSIT and / or WDM_STRICT_CFL (below) */
    /* Local self-interaction (Sec. 2.2, 2.4): the kick potential becomes
     * Phi + kappa |psi|^2 (kappa > 0 repulsive, < 0 attractive; 0 = none), the
     * energy gains kappa/2 int |psi|^4 and the CFL step a third term. */
    double kappa;
    /* Absorbing boundary (Sec. 3.1, Algorithm 1): after the second half kick
     * of every step psi <- psi * B, B = exp(-absorb_alpha dt sum_a g_a(x_a)),
     * g_a(x) = 2 - tanh(x / w_a) - tanh((L_a - x) / w_a), w_a = L_a /
     * absorb_nb, nodes x in [0, L).  absorb_alpha = 0 switches it off (the
     * paper's defaults are absorb_alpha = 10, absorb_nb = 50); absorb_nb > 0. */
    double absorb_alpha;
    double absorb_nb;
    /* Baryon treatment (Sec. 3.2.2): WDM_BARYON_DYNAMIC particles are kicked
     * and drift with the wave; WDM_BARYON_STATIC particles are deposited once
     * from the positions given to wdm_set_state and never move (their
     * velocities are kept as given). */
    int32_t baryon_mode;
    /* Particle leapfrog sub-steps per wave step (Sec. 3.2.2), 0 or 1 = one,
     * at most 1024.  The S sub-steps of h = dt / S run in the potential of the
     * step's start; the closing half kick takes the step's new potential, and
     * the baryons are deposited once, after the last sub-step. */
    int32_t nbody_substeps;
    /* Gravity boundary (Sec. 3.2.1): WDM_BOUNDARY_PERIODIC, the Fourier solve
     * with the mean removed; WDM_BOUNDARY_VACUUM, the isolated solve as a
     * convolution with the free-space Green's function -G dV / r on the
     * zero-padded (2 nx, 2 ny, 2 nz) grid (G = four_pi_G / (4 pi); the node's
     * own cell contributes -G h^2 C, C = 6 ln((1 + sqrt 3) / sqrt 2) - pi / 2,
     * the integral of 1/r over the unit cube).  Vacuum needs cubic cells and
     * n <= 256 per axis; the wave's own propagation stays periodic. */
    int32_t boundary;
    /* 1 reserves a per-member external (tidal) potential, set with
     * wdm_set_external_potential; 0 none. */
    int32_t external_potential;
} wdm_config;

/* Diagnostics of a synchronised state (Sec. 3.6 energy bookkeeping). */
typedef struct {
    double mass;               /* sum |psi|^2 dV */
    double e_kin;              /* eta^2/2 int |grad psi|^2, spectral */
    double e_pot;              /* 1/2 int (|psi|^2 + rho_b) Phi dV */
    double e_kin_particles;    /* 1/2 sum m v^2 */
    double e_total;            /* e_kin + e_pot + e_kin_particles + e_self */
    double momentum[3];        /* particle momentum sum m v */
    double max_abs_phi;        /* max |Phi| over the grid */
    double t;                  /* simulated time */
    double dt;                 /* time step last used (or selected) */
    double dt_auto;            /* CFL step of Sec. 3.5 from the last wdm_set_state */
    double e_self;             /* kappa/2 int |psi|^4 dV (included in e_total) */
    double max_rho;            /* max |psi|^2 over the grid */
    double e_ext;              /* int rho_tot Phi_ext dV of an external potential (in e_total;
                                  e_pot is then the self-gravity part, max_abs_phi and the
                                  CFL step are of the potential felt, self plus external) */
    double cfl_ratio;          /* largest |dt| / dt_max (Sec. 3.5) over the steps since the last
                                  wdm_set_state, dt_max from the potentials the steps' kicks
                                  used (see WDM_STRICT_CFL); 0 before the first step */
} wdm_energy_t;

/* The paper's diagnostics of a synchronised state (Sec. 3.6, App. A.1),
 * wave density only, second-order central differences on the periodic nodes. */
typedef struct {
    double K;                  /* 1/2 int |rho v|^2 / rho dV, rho v = eta Im(psi* grad psi)
                                  (cells with |psi|^2 <= 1e-30 skipped) */
    double Q;                  /* int |grad sqrt(rho)|^2 dV (as printed, without eta^2/2) */
    double V;                  /* int rho Phi dV (as printed, without 1/2) */
    double virial;             /* 2K + 2Q + V */
    double momentum[3];        /* wave momentum int rho v dV */
    double mass;               /* int |psi|^2 dV */
    double radii[9];           /* radii enclosing 10%, 20%, ..., 90% of the wave mass around
                                  the centre node: the smallest minimum-image node distance
                                  whose enclosed mass (nodes at that distance included)
                                  reaches the fraction; NaN unless the cells are cubic */
} wdm_diagnostics_t;

typedef struct {
    char name[40];             /* pass name, e.g. "x_kinetic" */
    int64_t launches;          /* launches recorded */
    double total_ms;           /* summed HIP-event durations */
} wdm_kernel_stat;

/* Bytes of device workspace a plan over `members` needs (256-byte aligned
 * sections).  Returns 0 for an invalid or unsupported configuration. */
size_t wdm_workspace_bytes(const wdm_config* members, int32_t n_members);

/* Create a plan for n_members boxes (n_members > 1: an ensemble advanced
 * together, one launch per pass per size class).  `workspace` is a device
 * buffer of at least wdm_workspace_bytes (caller owned, must outlive the
 * plan); `hip_stream` is the hipStream_t all work is ordered on (NULL = null
 * stream).  Twiddle tables are computed in FP64 on the host and uploaded
 * (this call synchronises).  *out receives the plan. */
wdm_status wdm_plan_create(const wdm_config* members, int32_t n_members, void* workspace,
                           size_t workspace_bytes, void* hip_stream, wdm_plan** out);
wdm_status wdm_plan_destroy(wdm_plan* plan);

/* Load the state of one member: psi (dev, [nx][ny][nz] complex of the plan
 * precision), pos and vel (dev, float [n_particles][3], may be NULL only when
 * n_particles == 0) at time t0.  Builds the initial potential Phi_0 from psi
 * and the deposited particles (Algorithm 1 needs Phi before its first kick),
 * its FP64 max |Phi| and the CFL step dt_auto of Sec. 3.5 (zeta = 0.9). */
wdm_status wdm_set_state(wdm_plan* plan, int32_t member, const void* psi, const float* pos,
                         const float* vel, double t0);

/* Per-member time step for ensembles, used by wdm_step(plan, n, 0). */
wdm_status wdm_set_member_dt(wdm_plan* plan, int32_t member, double dt);

/* Advance every member by n KDK steps (Eq. SPE_solver_KDK (a)-(d)).  dt != 0:
 * that step (negative = backwards in time) for all members; dt == 0: each
 * member's own dt (wdm_set_member_dt, else its dt_auto).  Half kicks of
 * consecutive steps share one potential and are merged.  The particle KDK
 * leapfrog is synchronous with the wave kicks (one particle step per wave
 * step).  Between calls the state is synchronised (positions, velocities and
 * psi at the same time). */
wdm_status wdm_step(wdm_plan* plan, int64_t n, double dt);

/* Copy psi (dev out, plan precision) of a member. */
wdm_status wdm_get_psi(wdm_plan* plan, int32_t member, void* psi_out);

/* Density |psi|^2, plus the CIC baryon density when include_baryons != 0
 * (dev out, real grid of the plan precision). */
wdm_status wdm_density(wdm_plan* plan, int32_t member, void* rho_out, int32_t include_baryons);

/* Total potential Phi of the synchronised state (dev out, real grid). */
wdm_status wdm_potential(wdm_plan* plan, int32_t member, void* phi_out);

/* FP64 diagnostics (host out).  Synchronises the plan's stream.  Returns
 * WDM_EUNSTABLE, leaving *out untouched, when the state or a step's potential
 * was non-finite, or (WDM_STRICT_CFL) a step exceeded the CFL bound. */
wdm_status wdm_energy(wdm_plan* plan, int32_t member, wdm_energy_t* out);

/* External (tidal) potential of a member created with external_potential =
 * 1 (Sec. 4.3): phi_ext (dev, real [nx][ny][nz] of the plan precision; NULL
 * = zero) is copied, and its mean acceleration removed: along each axis the
 * gradient averaged over the nodes symmetric about the centre node (1 .. n-1,
 * the other two axes over all nodes), (phi[n-1] - phi[1]) / ((n - 2) h), is
 * subtracted as a ramp through the box centre.  The corrected potential is
 * added to the self-gravity felt by the wave and the particles from the next
 * step on (set it before wdm_set_state for dt_auto to include it).  For a
 * time-dependent field, set it again between wdm_step calls. */
wdm_status wdm_set_external_potential(wdm_plan* plan, int32_t member, const void* phi_ext);

/* The paper's halo diagnostics (host out): K, Q, V, 2K + 2Q + V, the wave
 * momentum and mass, and the mass-fraction radii around the node centre[3]
 * (NULL = (nx/2, ny/2, nz/2), the box centre; each index in [0, n)).  V uses
 * the potential of the synchronised state.  Uses the plan's shared scratch;
 * synchronises the plan's stream.  FP64 sums; K, Q, V and the momentum are
 * deterministic, the radial histogram uses FP64 atomics (last bits only). */
wdm_status wdm_diagnostics(wdm_plan* plan, int32_t member, const int32_t* centre,
                           wdm_diagnostics_t* out);

/* Particle positions and velocities in their original order (dev out,
 * float [n_particles][3]; either pointer may be NULL). */
wdm_status wdm_particles(wdm_plan* plan, int32_t member, float* pos_out, float* vel_out);

/* Forward (inverse = 0, unnormalised exp(-i k.x)) or inverse (inverse = 1,
 * scaled by 1/N) 3D FFT of a member's psi in place -- the transform used by
 * the drift step (b) -- exposed for verification.  Leaves the member's
 * state unsynchronised: call wdm_set_state before stepping again. */
wdm_status wdm_fft3d(wdm_plan* plan, int32_t member, int32_t inverse);

/* Allocation-free variant of wdm_fft3d, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same 3D transform of a caller's buffer, with no
 * plan and no workspace.  psi_in and psi_out (dev, [nx][ny][nz] complex64 for
 * precision WDM_C64, complex128 for WDM_C128) may be the same buffer (in
 * place) or must not overlap; psi_in is read, psi_out receives the forward
 * (inverse = 0, unnormalised exp(-i k.x)) or inverse (inverse = 1, scaled by
 * 1/N) transform; stream-ordered on hip_stream (NULL = null stream).
 * Axis lengths as for wdm_config (at most 512 per axis).  The library's only
 * device memory for it is a fixed 32 KB array per GPU (the descriptor and the
 * three twiddle tables, rewritten by every call), held until the process
 * ends; the first call on a device looks up that array's address, so make it
 * once outside any capture.  It calls no hipMalloc or hipFree.  All calls on
 * one GPU share the array: calls that overlap in time on one GPU (on
 * different streams, or from different threads) race and must be ordered by
 * the caller.  Returns WDM_EUNSUPPORTED for other axis lengths, WDM_EINVAL
 * for null pointers or a bad precision; nothing is launched then. */
wdm_status wdm_fft3d_noalloc(const void* psi_in, void* psi_out, int32_t nx, int32_t ny, int32_t nz,
                             int32_t precision, int32_t inverse, void* hip_stream);

/* Replay captured HIP graphs of the merged step (default on).  Off: every
 * kernel is launched directly on the plan's stream.  Results are the same
 * either way; profiling always launches directly. */
wdm_status wdm_use_graphs(wdm_plan* plan, int32_t enable);

/* Re-sort particles by cell every `interval` steps (0 = only in
 * wdm_set_state).  Ordering only affects speed and atomic summation order. */
wdm_status wdm_set_sort_interval(wdm_plan* plan, int32_t interval);

/* Autotuning of the step's FFT passes.  Each tunable pass (P1, P2/P4, P3, P5,
 * P6/P8, P7) of each size class chooses among up to four FFT plans: 0, the
 * default; 1, where the axis length allows (32, 64, 128, 256, 384, 512), twice
 * the lanes per pencil and half the values per lane; 2, for the strided
 * passes (P2/P4, P3, P6/P8, P7) at axis lengths up to 256, the default radices
 * with twice the pencils per work-group (256-byte row segments for complex64,
 * the "z-chunk width"); 3, the default radices exchanging whole complex
 * values through LDS (one barrier pair per radix level instead of two, twice
 * the LDS), for the strided passes at axis lengths up to 256 and for the z
 * passes at 16, 32, 64, 128 and 256 (whose default splits the exchange).
 * wdm_autotune times the available plans on the plan's
 * stream (a warm-up launch each, then `reps` rounds, reps in [1, 1000], timing
 * each plan once per round in rotating order, each launch between its own
 * events, on zeroed fields) and leaves the default unless another plan's
 * median is at least 2 % below the default's (then the fastest such plan).
 * It overwrites the members' states: call it before wdm_set_state, or set
 * every state again afterwards (wdm_step returns WDM_ESTATE until then).
 * Synchronises.  All plans give the same results up to rounding.
 *
 * wdm_tuning_entries: number of int32 entries of the choice table (size
 * classes in ascending (nx, ny, nz) order, six passes each in the order above;
 * 0 for a null plan).  wdm_get_tuning / wdm_set_tuning copy the table to / from
 * a host array of exactly that length (values 0 to 3, each only where that
 * plan exists for the pass and its axis length, else WDM_EINVAL and nothing
 * changes), e.g. to reuse a cached choice without re-timing. */
wdm_status wdm_autotune(wdm_plan* plan, int32_t reps);
int32_t wdm_tuning_entries(const wdm_plan* plan);
wdm_status wdm_get_tuning(wdm_plan* plan, int32_t* out, int32_t n);
wdm_status wdm_set_tuning(wdm_plan* plan, const int32_t* in, int32_t n);

/* Per-pass timing: while enabled, every kernel launch of wdm_step is
 * bracketed by HIP events on the plan's stream.  wdm_profile_read
 * synchronises, reports one entry per pass (up to `cap`, host array) and
 * clears the record. */
wdm_status wdm_profile(wdm_plan* plan, int32_t enable);
wdm_status wdm_profile_read(wdm_plan* plan, wdm_kernel_stat* out, int32_t cap, int32_t* count);

/* Achievable-bandwidth reference: a plain float4 copy of `bytes` from src to
 * dst (dev), `reps` times on `hip_stream`; returns the mean ms per copy
 * (host out).  Synchronises. */
wdm_status wdm_copy_bandwidth(void* dst, const void* src, size_t bytes, int32_t reps,
                              void* hip_stream, double* ms_per_copy);

/* ---- spectral utilities of the learned-corrector workload --------------
 * Not part of the paper's method: they serve the corrector's training-pair
 * generation (restriction) and its P(k) judge. */

/* Spectral restriction of a fine member's psi to the coarse member's grid
 * (cubic grids, same box, nc < nf): keep the modes with |m_i| < nc/2 on every
 * axis (the coarse Nyquist planes are dropped) so point values of
 * band-limited fields are preserved; write the coarse field to psi_out (dev,
 * nc^3 complex of the plans' precision).  Both plans must share a stream.  Uses
 * both plans' scratch space. */
wdm_status wdm_restrict(wdm_plan* fine, int32_t fine_member, wdm_plan* coarse,
                        int32_t coarse_member, void* psi_out);

/* Shell power spectrum of the density contrast delta = |psi|^2 / mean - 1 on a
 * cubic grid: shell b = round(|m|) (integer mode vector m), pk[b] = mean over
 * the shell of |delta_k|^2 / N^2 (N = n^3), counts[b] = modes in the shell
 * (host out, nbins entries each; counts may be NULL).  FP64 sums.
 * Synchronises. */
wdm_status wdm_power_spectrum(wdm_plan* plan, int32_t member, int32_t nbins, double* pk,
                              int64_t* counts);

/* Field distance for the corrector's judge: out[0] = sum |psi - other|^2,
 * out[1] = sum |other|^2 over the member's grid (other: dev, same shape and
 * precision as psi), FP64 sums in a fixed order (host out; synchronises). */
wdm_status wdm_distance(wdm_plan* plan, int32_t member, const void* other, double* out);

/* ---- learned corrector ----------------------------------------------------
 * Not part of the paper's method: a network that corrects a 2x-coarser
 * split-step run toward the fine one every few coarse steps.
 * A three-layer 3x3x3 convolution network on an n^3 periodic grid:
 * 3 -> 16 (ReLU) -> 16 (ReLU) -> 2 channels, circular padding.  Weights and
 * activations are BF16 on the matrix cores with FP32 accumulation; FP32
 * master parameters, gradients and Adam moments live in the network
 * workspace.  Parameter vector layout (wdm_net_param_count floats), per layer
 * l in order: w_l[cout][cin][27] then b_l[cout], tap index
 * (dx+1)*9 + (dy+1)*3 + (dz+1) for neighbour (i+dx, j+dy, k+dz).  Inputs are
 * f32 [n^3][3], outputs f32 [n^3][2] (channels last, C order cells). */
typedef struct wdm_net wdm_net;

int32_t wdm_net_param_count(void);
size_t wdm_net_workspace_bytes(int32_t n);
/* Parameters start at zero; set them with wdm_net_set_params. */
wdm_status wdm_net_create(int32_t n, void* workspace, size_t workspace_bytes, void* hip_stream,
                          wdm_net** out);
wdm_status wdm_net_destroy(wdm_net* net);
/* Host in / out, synchronous; set_params also resets the Adam state. */
wdm_status wdm_net_set_params(wdm_net* net, const float* params);
wdm_status wdm_net_get_params(wdm_net* net, float* params);
wdm_status wdm_net_get_grads(wdm_net* net, float* grads);
/* Forward pass; keeps the activations for a following backward pass.  y may
 * be NULL (output kept internally). */
wdm_status wdm_net_forward(wdm_net* net, const float* x, float* y);
/* Backward pass from dL/dy (dev f32 [n^3][2]) of the last forward pass:
 * overwrites the parameter gradients. */
wdm_status wdm_net_backward(wdm_net* net, const float* dy);
/* Mean-squared error of the last forward output against target (dev f32
 * [n^3][2]), its backward pass, and the loss (host out, may be NULL;
 * synchronises when given). */
wdm_status wdm_net_mse_backward(wdm_net* net, const float* target, double* loss);
/* One Adam step on the FP32 master parameters (bias-corrected). */
wdm_status wdm_net_adam(wdm_net* net, double lr, double b1, double b2, double eps);
/* Normalisation held by the network (device scalars; all 1 at creation):
 * inputs enter as (Re psi s_psi, Im psi s_psi, Phi s_phi), the network learns
 * residuals divided by s_out (wdm_net_mse_backward compares its output with
 * target / s_out) and a correction adds s_out times its output.  The forward
 * pass scales its caller inputs x the same way. */
wdm_status wdm_net_set_scales(wdm_net* net, double s_psi, double s_phi, double s_out);
/* out[3] = (s_psi, s_phi, s_out) (host out; synchronises). */
wdm_status wdm_net_get_scales(wdm_net* net, double* out);
/* Scales from a training set of `count` pairs (host arrays of device
 * pointers to wdm_net_pair outputs of the network's grid): s_psi = 1 / rms
 * |psi|, s_phi = 1 / std(Phi), s_out = std of the residual's components
 * (population moments, FP64 deterministic sums). */
wdm_status wdm_net_fit_scales(wdm_net* net, const float* const* xs, const float* const* ys,
                              int32_t count);
/* A training pair from a complex64 member's synchronised state and a target
 * field of the same grid (dev, complex64): x_out = (Re psi, Im psi, Phi) as f32
 * [n^3][3], y_out = target - psi as f32 [n^3][2] (dev outs, channels last). */
wdm_status wdm_net_pair(wdm_plan* plan, int32_t member, const void* target, float* x_out,
                        float* y_out);
/* Apply the corrector to a complex64 member of the network's grid: inputs
 * from (psi, Phi) with the network's scales, psi += s_out * output, psi
 * rescaled to its FP64 mass before the correction, and the potential rebuilt
 * from the corrected state (moving particles redeposited), so the state is
 * synchronised again.  The network and the plan must share a stream. */
wdm_status wdm_net_apply(wdm_net* net, wdm_plan* plan, int32_t member);
/* Attach the corrector to a plan: from now on wdm_step applies it to
 * `member` after every `every` steps (counted across calls; 1 <= every <=
 * 4096), as wdm_net_apply would between calls.  A run of `every` steps that
 * starts at a correction boundary replays one captured graph holding the
 * steps, the closing half kick and the correction.  net = NULL or every = 0
 * detaches.  The network must stay alive while attached. */
wdm_status wdm_plan_attach_corrector(wdm_plan* plan, wdm_net* net, int32_t member,
                                     int32_t every);

/* Message for the last failing call on this thread ("" if none). */
const char* wdm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* WDM_H */
