/*
 * FP64 CPU oracle for the Schroedinger-Poisson kick-drift-kick split step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Conventions (readings of the paper, Sec. 3.1 - 3.5):
 *   - periodic box, node-centred grid x_i = i * dx, dx = L / n (the paper's
 *     L/(N-1) would make both box ends the same periodic point);
 *   - arrays are C-ordered [nx][ny][nz], z contiguous; complex values are
 *     interleaved (re, im) doubles;
 *   - forward DFT is unnormalised with exp(-i k.x); the inverse carries 1/N;
 *   - wave numbers k_m = 2 pi m / L with m in {0..n/2-1, -n/2..-1} (Nyquist
 *     kept with k^2 = (pi n / L)^2), continuous |k|^2 Laplacian symbol;
 *   - eta = hbar/m; kick exp(-i Phi tau / eta), drift exp(-i eta |k|^2 dt / 2);
 *   - Poisson: Phi_k = -(4 pi G) rho_k / |k|^2, k = 0 mode set to zero.
 */
#ifndef WDM_ORACLE_H
#define WDM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz;
    double lx, ly, lz;
    double hbar_over_m;     /* eta */
    double four_pi_G;       /* 0 switches gravity off (free Schroedinger) */
    int64_t n_particles;
    double particle_mass;   /* equal-mass particles */
    /* local self-interaction (Sec. 2.2, 2.4): the kick potential is
     * Phi + kappa |psi|^2; 0 = non-interacting */
    double kappa;
    /* absorbing boundary mask (Sec. 3.1, Algorithm 1): after the second half
     * kick of every step psi <- psi * B(x), B = exp(-alpha dt sum_a g_a(x_a)),
     * g_a(x) = 2 - tanh(x / w_a) - tanh((L_a - x) / w_a), w_a = L_a / n_b;
     * alpha = 0 switches it off */
    double absorb_alpha;
    double absorb_nb;
    /* baryon treatment (Sec. 3.2.2): 0 dynamic particles, 1 static particles
     * (deposited from their fixed positions, never kicked or moved) */
    int32_t baryon_mode;
    /* particle leapfrog sub-steps per wave step (0 or 1: one).  The S
     * sub-steps of h = dt / S run in the potential of the step's start; the
     * last half kick takes the step's new potential */
    int32_t nbody_substeps;
    /* gravity boundary: 0 periodic (Fourier solve, mean removed), 1 vacuum
     * (isolated solve by zero-padded convolution; cubic cells) */
    int32_t boundary;
} orc_config;

/* Number of worker threads (0 = all hardware threads).  Results never depend
 * on it: work is split over independent pencils/particles only and every sum
 * is taken in a fixed order.  Returns the count now in use. */
int orc_set_threads(int n);
int orc_get_threads(void);

/* 1D and 3D FFTs over interleaved complex doubles.  sign = -1: forward,
 * unnormalised; sign = +1: inverse, scaled by 1/n (per axis).  Lengths must be
 * 2^a 3^b.  Returns 0, or -1 for an unsupported length. */
int orc_fft1d(double* data, int n, int sign);
int orc_fft3d(double* data, int nx, int ny, int nz, int sign);
/* Brute-force O(N^2) 3D DFT straight from the definition (same conventions). */
void orc_dft3d_brute(const double* in, double* out, int nx, int ny, int nz, int sign);

/* Periodic FFT Poisson solve: phi = F^-1[-(4 pi G)/|k|^2 F rho], k=0 -> 0. */
void orc_poisson(const orc_config* c, const double* rho, double* phi);
/* CIC deposit of all particles into rho_b (overwritten), density units m/dx^3. */
void orc_cic_deposit(const orc_config* c, const double* pos, double* rho_b);
/* g = -grad(phi) by 2nd-order central differences at nodes, CIC-interpolated
 * to the particle positions.  acc is [Np][3]. */
void orc_cic_force(const orc_config* c, const double* phi, const double* pos, double* acc);
/* Total potential of the state: Poisson(|psi|^2 + CIC(pos)). */
void orc_potential(const orc_config* c, const double* psi, const double* pos, double* phi);

/* Advance psi (complex [nx][ny][nz]) and particles (pos, vel [Np][3], may be
 * NULL when n_particles == 0) by nsteps unmerged KDK steps of size dt (dt may
 * be negative).  The starting potential is rebuilt from the state.  Particles
 * take nbody_substeps leapfrog sub-steps per step; static particles
 * (baryon_mode 1) are left untouched. */
void orc_kdk(const orc_config* c, double* psi, double* pos, double* vel, int64_t nsteps,
             double dt);

/* orc_kdk with an external potential phi_ext (real [nx][ny][nz], already
 * corrected by orc_tidal_correct; NULL = none) added to the self-gravity felt
 * by the wave and the particles. */
void orc_kdk_ext(const orc_config* c, double* psi, double* pos, double* vel, int64_t nsteps,
                 double dt, const double* phi_ext);

/* Isolated Poisson solve by direct summation over all node pairs with the
 * same sampled Green's function (O(N^6): small grids only). */
void orc_poisson_direct(const orc_config* c, const double* rho, double* phi);
/* The same sum at `count` listed nodes (i, j, k triples in `nodes`); phi[count]. */
void orc_poisson_direct_at(const orc_config* c, const double* rho, const int64_t* nodes,
                           int64_t count, double* phi);
/* Integral of 1/|u| over the unit cube centred at the origin. */
double orc_cube_self_integral(void);
/* External (tidal) potential with its mean acceleration removed (Sec. 4.3). */
void orc_tidal_correct(const orc_config* c, const double* phi_in, double* phi_out);

/* Energies of a synchronised state.  out[0..10] =
 *   mass = sum |psi|^2 dV, e_kin (spectral, eta^2/2 int |grad psi|^2),
 *   e_pot = 1/2 int rho_tot Phi dV, e_kin_particles = 1/2 sum m v^2,
 *   e_total (including e_self), momentum of the particles (3), max |Phi|,
 *   e_self = kappa/2 int |psi|^4 dV, max |psi|^2. */
void orc_energy(const orc_config* c, const double* psi, const double* pos, const double* vel,
                double* out);
/* orc_energy with an external potential: out[11] = int rho_tot phi_ext dV
 * (in e_total; max |Phi| is of the potential felt, self plus external). */
void orc_energy_ext(const orc_config* c, const double* psi, const double* pos, const double* vel,
                    const double* phi_ext, double* out);
/* The paper's overall energy terms (Sec. 3.6) exactly as printed:
 *   out[0] K = 1/2 int |rho v|^2 / rho (rho v = eta Im(psi* grad psi), central
 *              differences, cells with rho <= 1e-30 skipped),
 *   out[1] Q = int |grad sqrt(rho)|^2 (central differences),
 *   out[2] V = int rho Phi,   out[3] 2K + 2Q + V,
 *   out[4..6] wave momentum int rho v.  Wave density only. */
void orc_paper_energies(const orc_config* c, const double* psi, const double* phi, double* out);

/* Mass-fraction radii (App. A.1.2) of the wave mass around the node
 * centre[3]: radii[f] = smallest minimum-image node distance whose enclosed
 * mass reaches fractions[f] of the total.  Needs cubic cells (returns -1
 * otherwise, 0 on success). */
int orc_mass_fraction_radii(const orc_config* c, const double* psi, const int32_t* centre,
                            const double* fractions, int nf, double* radii);

/* dt = zeta * 0.5 * min{c_kin dx_min^2 / eta, 2 pi eta / max|phi|,
 *                       2 pi eta / (|kappa| max|psi|^2)} (Sec. 3.5); psi may be
 * NULL when kappa = 0. */
double orc_dt_auto(const orc_config* c, const double* phi, const double* psi, double zeta,
                   double c_kin);
/* The absorbing mask B of one step of size dt, real [nx][ny][nz]. */
void orc_absorb_mask(const orc_config* c, double dt, double* mask);

/* Shell power spectrum of delta = rho/mean(rho) - 1 (rho real [n]^3, cubic
 * grid): shell b = round(|m|); pk[b] = mean over the shell of |delta_k|^2 / N^2
 * (N = n^3), counts[b] = modes in the shell; nbins entries. */
void orc_power_spectrum(const double* rho, int n, int nbins, double* pk, int64_t* counts);
/* Spectral restriction of a complex field from nf^3 to nc^3 (nc < nf): keep
 * modes with |m_i| < nc/2 on every axis (coarse Nyquist dropped), preserving
 * point values (coefficients scaled by nc^3/nf^3). */
void orc_restrict(const double* fine, int nf, double* coarse, int nc);

/* ---- 3D convolution corrector (FP64, weights/activations rounded to bf16) ----
 * Layer l maps cin -> cout channels with a 3x3x3 kernel, circular padding,
 * bias, ReLU after every layer but the last.  x is [cin][n][n][n] (fp64 values
 * that the caller has already rounded as it wishes); w is [cout][cin][3][3][3]
 * with tap index (dx+1)*9+(dy+1)*3+(dz+1) for neighbour (i+dx, j+dy, k+dz).
 * y[co][p] = b[co] + sum_{ci,tap} w[co][ci][tap] * x[ci][p + tap]. */
void orc_conv3d_fwd(const double* x, const double* w, const double* b, double* y,
                    int n, int cin, int cout);
/* Backward of the same conv: given dy, accumulate dx (if non-NULL, overwritten),
 * dw and db (overwritten). */
void orc_conv3d_bwd(const double* x, const double* w, const double* dy, double* dx,
                    double* dw, double* db, int n, int cin, int cout);
/* Round-to-nearest-even to bfloat16 and back, element-wise, in place. */
void orc_round_bf16(double* v, int64_t count);

#ifdef __cplusplus
}
#endif
#endif
