// The Schroedinger-Poisson split step of the oracle, taken step by step from
// the paper: the kick-drift-kick sequence of Eq. (SPE_solver_KDK) and
// Algorithm 1 (Sec. 3.1), the periodic FFT Poisson solver (Sec. 3.2.1), the
// second-order central-difference gradient (Sec. 3.1), the dynamic two-way
// particle coupling (Sec. 3.2.2, here through the mesh with cloud-in-cell
// weights) and the CFL time step (Sec. 3.5).  Plain FP64, no fusion.
#include <cmath>
#include <cstring>

#include "common.hpp"

namespace orc {

struct Grid {
    int64_t nx, ny, nz;
    double lx, ly, lz, dx, dy, dz, dv;
    explicit Grid(const orc_config* c)
        : nx(c->nx), ny(c->ny), nz(c->nz), lx(c->lx), ly(c->ly), lz(c->lz) {
        dx = lx / nx;
        dy = ly / ny;
        dz = lz / nz;
        dv = dx * dy * dz;
    }
    int64_t n() const { return nx * ny * nz; }
    int64_t at(int64_t i, int64_t j, int64_t k) const {
        return (wrap_index(i, nx) * ny + wrap_index(j, ny)) * nz + wrap_index(k, nz);
    }
    // |k|^2 of the mode stored at (i, j, k)
    double k2(int64_t i, int64_t j, int64_t k) const {
        const double kx = kTwoPi * double(signed_mode(i, nx)) / lx;
        const double ky = kTwoPi * double(signed_mode(j, ny)) / ly;
        const double kz = kTwoPi * double(signed_mode(k, nz)) / lz;
        return kx * kx + ky * ky + kz * kz;
    }
};

// Integral of 1/|u| over the unit cube centred on u = 0.  Split into the six
// pyramids on which one coordinate is largest; in each, u = x (1, s, t) gives
// 6 * int_0^(1/2) x dx * int int_[-1,1]^2 (1 + s^2 + t^2)^(-1/2) ds dt
// = (3/4) * 4 * J, J = int int_[0,1]^2 (1 + s^2 + t^2)^(-1/2), the smooth J
// taken by 24-point Gauss-Legendre in each variable (nodes by Newton on P_24).
static double cube_self_integral() {
    const int m = 24;
    double xs[m], ws[m];
    for (int i = 0; i < m; ++i) {
        double x = std::cos(kPi * (i + 0.75) / (m + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= m; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = m * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        xs[i] = 0.5 * (x + 1.0);              // mapped to [0, 1]
        ws[i] = 1.0 / ((1.0 - x * x) * dp * dp);  // 2/((1-x^2)P'^2), halved
    }
    double J = 0.0;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j)
            J += ws[i] * ws[j] / std::sqrt(1.0 + xs[i] * xs[i] + xs[j] * xs[j]);
    return 3.0 * J;
}

// Sampled free-space Green's function of the isolated solve (Sec. 3.2.1,
// vacuum boundary): g(r) = -G dV / |r| between nodes, and for the node itself
// -G times the integral of 1/|x| over its own cell (cubic cells, h^2 times the
// unit-cube integral), G = four_pi_G / (4 pi).
static double green_iso(const orc_config* c, const Grid& g, int64_t di, int64_t dj, int64_t dk,
                        double self) {
    const double G = c->four_pi_G / (4.0 * kPi);
    if (di == 0 && dj == 0 && dk == 0) return -G * g.dx * g.dx * self;
    const double x = di * g.dx, y = dj * g.dy, z = dk * g.dz;
    return -G * g.dv / std::sqrt(x * x + y * y + z * z);
}

// Isolated Poisson solve: the linear convolution Phi = g * rho over the box,
// as a circular convolution on the zero-padded (2 nx, 2 ny, 2 nz) grid (the
// O(N^3 log N) stand-in for the O(N^4) method the paper cites).
static void poisson_isolated(const orc_config* c, const double* rho, double* phi) {
    Grid g(c);
    const int64_t px = 2 * g.nx, py = 2 * g.ny, pz = 2 * g.nz, pn = px * py * pz;
    const double self = cube_self_integral();
    std::vector<cplx> fr(size_t(pn), cplx(0.0, 0.0));
    std::vector<cplx> fg(static_cast<size_t>(pn));
    for (int64_t i = 0; i < g.nx; ++i)
        for (int64_t j = 0; j < g.ny; ++j)
            for (int64_t k = 0; k < g.nz; ++k)
                fr[size_t((i * py + j) * pz + k)] = cplx(rho[(i * g.ny + j) * g.nz + k], 0.0);
    for (int64_t i = 0; i < px; ++i)
        for (int64_t j = 0; j < py; ++j)
            for (int64_t k = 0; k < pz; ++k) {
                // offsets of the padded circulant: i and i - 2n are the same node
                const int64_t di = i <= g.nx ? i : i - px, dj = j <= g.ny ? j : j - py,
                              dk = k <= g.nz ? k : k - pz;
                fg[size_t((i * py + j) * pz + k)] = cplx(green_iso(c, g, di, dj, dk, self), 0.0);
            }
    fft3d(fr.data(), int(px), int(py), int(pz), -1);
    fft3d(fg.data(), int(px), int(py), int(pz), -1);
    for (int64_t q = 0; q < pn; ++q) fr[size_t(q)] *= fg[size_t(q)];
    fft3d(fr.data(), int(px), int(py), int(pz), +1);
    for (int64_t i = 0; i < g.nx; ++i)
        for (int64_t j = 0; j < g.ny; ++j)
            for (int64_t k = 0; k < g.nz; ++k)
                phi[(i * g.ny + j) * g.nz + k] = fr[size_t((i * py + j) * pz + k)].real();
}

// (c) Phi = F^-1{ -(4 pi G) / k^2 F{rho} }, mean removed by zeroing k = 0;
// with the vacuum boundary the isolated solve above.
static void poisson(const orc_config* c, const double* rho, double* phi) {
    if (c->boundary == 1) {
        poisson_isolated(c, rho, phi);
        return;
    }
    Grid g(c);
    std::vector<cplx> f(g.n());
    for (int64_t i = 0; i < g.n(); ++i) f[i] = cplx(rho[i], 0.0);
    fft3d(f.data(), int(g.nx), int(g.ny), int(g.nz), -1);
    parallel_for(g.nx, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i)
            for (int64_t j = 0; j < g.ny; ++j)
                for (int64_t k = 0; k < g.nz; ++k) {
                    const int64_t o = (i * g.ny + j) * g.nz + k;
                    const double k2 = g.k2(i, j, k);
                    f[o] = (i == 0 && j == 0 && k == 0) ? cplx(0.0, 0.0)
                                                        : f[o] * (-c->four_pi_G / k2);
                }
    });
    fft3d(f.data(), int(g.nx), int(g.ny), int(g.nz), +1);
    for (int64_t i = 0; i < g.n(); ++i) phi[i] = f[i].real();
}

// Cloud-in-cell: s = x/dx, cell i = floor(s), f = s - i, weights (1-f, f) per
// axis on nodes i and i+1 (periodic).
struct Cic {
    int64_t i[3];
    double w[3][2];
};

static Cic cic_of(const Grid& g, const double* p) {
    Cic r;
    const double h[3] = {g.dx, g.dy, g.dz};
    for (int a = 0; a < 3; ++a) {
        const double s = p[a] / h[a];
        const double fl = std::floor(s);
        const double f = s - fl;
        r.i[a] = int64_t(fl);
        r.w[a][0] = 1.0 - f;
        r.w[a][1] = f;
    }
    return r;
}

static void cic_deposit(const orc_config* c, const double* pos, double* rho_b) {
    Grid g(c);
    std::fill(rho_b, rho_b + g.n(), 0.0);
    const double q = c->particle_mass / g.dv;
    for (int64_t p = 0; p < c->n_particles; ++p) {  // sequential, fixed order
        Cic w = cic_of(g, pos + 3 * p);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int d = 0; d < 2; ++d)
                    rho_b[g.at(w.i[0] + a, w.i[1] + b, w.i[2] + d)] +=
                        q * (w.w[0][a] * w.w[1][b] * w.w[2][d]);
    }
}

// g = -grad(Phi) at node (i,j,k) by central differences.
static void node_accel(const Grid& g, const double* phi, int64_t i, int64_t j, int64_t k,
                       double* out) {
    out[0] = -(phi[g.at(i + 1, j, k)] - phi[g.at(i - 1, j, k)]) / (2.0 * g.dx);
    out[1] = -(phi[g.at(i, j + 1, k)] - phi[g.at(i, j - 1, k)]) / (2.0 * g.dy);
    out[2] = -(phi[g.at(i, j, k + 1)] - phi[g.at(i, j, k - 1)]) / (2.0 * g.dz);
}

static void cic_force(const orc_config* c, const double* phi, const double* pos, double* acc) {
    Grid g(c);
    parallel_for(c->n_particles, [&](int64_t b0, int64_t e0) {
        for (int64_t p = b0; p < e0; ++p) {
            Cic w = cic_of(g, pos + 3 * p);
            double s[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    for (int d = 0; d < 2; ++d) {
                        double na[3];
                        node_accel(g, phi, w.i[0] + a, w.i[1] + b, w.i[2] + d, na);
                        const double wt = w.w[0][a] * w.w[1][b] * w.w[2][d];
                        for (int t = 0; t < 3; ++t) s[t] += wt * na[t];
                    }
            for (int t = 0; t < 3; ++t) acc[3 * p + t] = s[t];
        }
    });
}

static void total_potential(const orc_config* c, const cplx* psi, const double* pos,
                            double* phi) {
    Grid g(c);
    std::vector<double> rho(g.n(), 0.0);
    if (c->n_particles > 0) cic_deposit(c, pos, rho.data());
    for (int64_t i = 0; i < g.n(); ++i) rho[i] += std::norm(psi[i]);
    poisson(c, rho.data(), phi);
}

// (a)/(d): psi <- exp(-i V tau / eta) psi with V = Phi + kappa |psi|^2 (the
// local self-interaction of Sec. 2.2 / 2.4 as an extra potential; the kick
// keeps |psi|, so V taken at its start is exact).
static void kick(const orc_config* c, cplx* psi, const double* phi, double tau) {
    const int64_t n = cells(c);
    const double s = tau / c->hbar_over_m;
    const double kappa = c->kappa;
    parallel_for(n, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
            const double v = phi[i] + kappa * std::norm(psi[i]);
            psi[i] *= std::polar(1.0, -v * s);
        }
    });
}

// Absorbing boundary profile of one axis (Sec. 3.1) at node x in [0, L): zero
// in the interior, 1 at the faces.  The paper's nodes run from -L/2, ours from
// 0: its x +- L/2 are our x and x - L.
static double absorb_profile(double x, double L, double nb) {
    const double w = L / nb;
    return 2.0 - std::tanh(x / w) + std::tanh((x - L) / w);
}

// B(x) = exp(-alpha dt sum_a g_a(x_a)) on the nodes.
static void absorb_mask(const orc_config* c, double dt, double* mask) {
    Grid g(c);
    for (int64_t i = 0; i < g.nx; ++i)
        for (int64_t j = 0; j < g.ny; ++j)
            for (int64_t k = 0; k < g.nz; ++k) {
                const double s = absorb_profile(double(i) * g.dx, g.lx, c->absorb_nb) +
                                 absorb_profile(double(j) * g.dy, g.ly, c->absorb_nb) +
                                 absorb_profile(double(k) * g.dz, g.lz, c->absorb_nb);
                mask[(i * g.ny + j) * g.nz + k] = std::exp(-c->absorb_alpha * dt * s);
            }
}

// (b): psi <- F^-1{ exp(-i eta k^2 dt / 2) F{psi} }.
static void drift(const orc_config* c, cplx* psi, double dt) {
    Grid g(c);
    fft3d(psi, int(g.nx), int(g.ny), int(g.nz), -1);
    parallel_for(g.nx, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i)
            for (int64_t j = 0; j < g.ny; ++j)
                for (int64_t k = 0; k < g.nz; ++k)
                    psi[(i * g.ny + j) * g.nz + k] *=
                        std::polar(1.0, -0.5 * c->hbar_over_m * g.k2(i, j, k) * dt);
    });
    fft3d(psi, int(g.nx), int(g.ny), int(g.nz), +1);
}

static void particle_kick(const orc_config* c, const double* phi, const double* pos,
                          double* vel, double tau, std::vector<double>& acc) {
    acc.resize(size_t(3 * c->n_particles));
    cic_force(c, phi, pos, acc.data());
    for (int64_t i = 0; i < 3 * c->n_particles; ++i) vel[i] += acc[i] * tau;
}

static void particle_drift(const orc_config* c, double* pos, const double* vel, double dt) {
    const double L[3] = {c->lx, c->ly, c->lz};
    for (int64_t p = 0; p < c->n_particles; ++p)
        for (int a = 0; a < 3; ++a) {
            double x = pos[3 * p + a] + vel[3 * p + a] * dt;
            x -= L[a] * std::floor(x / L[a]);
            if (x >= L[a]) x = 0.0;
            pos[3 * p + a] = x;
        }
}

// Particle part of one wave step with S leapfrog sub-steps of h = dt / S
// (Sec. 3.2.2: the N-body component advances in several sub-steps per wave
// step).  The grid potential is that of the step's start for every sub-step;
// the closing half kick, after the step's Poisson solve, is done by the caller.
static void particle_substeps(const orc_config* c, const double* phi, double* pos, double* vel,
                              double dt, std::vector<double>& acc) {
    const int S = c->nbody_substeps > 1 ? c->nbody_substeps : 1;
    const double h = dt / S;
    for (int k = 0; k < S; ++k) {
        particle_kick(c, phi, pos, vel, 0.5 * h, acc);
        particle_drift(c, pos, vel, h);
        if (k + 1 < S) particle_kick(c, phi, pos, vel, 0.5 * h, acc);
    }
}

// Potential felt by the wave and the particles: self-gravity plus the
// (already corrected) external potential, if any.
static void add_external(const orc_config* c, const double* phi_ext, double* phi) {
    if (!phi_ext) return;
    for (int64_t i = 0; i < cells(c); ++i) phi[i] += phi_ext[i];
}

static void kdk(const orc_config* c, cplx* psi, double* pos, double* vel, int64_t nsteps,
                double dt, const double* phi_ext) {
    const int64_t n = cells(c);
    // static baryons (Sec. 3.2.2) only source the potential
    const bool parts = c->n_particles > 0 && c->baryon_mode == 0;
    const int S = c->nbody_substeps > 1 ? c->nbody_substeps : 1;
    std::vector<double> phi(n), acc, mask;
    if (c->absorb_alpha != 0.0) {
        mask.resize(size_t(n));
        absorb_mask(c, dt, mask.data());
    }
    total_potential(c, psi, pos, phi.data());
    add_external(c, phi_ext, phi.data());
    for (int64_t s = 0; s < nsteps; ++s) {
        // (a) first half kick with the current potential
        kick(c, psi, phi.data(), 0.5 * dt);
        // particles: first half kick and drift (one sub-step), or all but the
        // last half kick of S sub-steps in the potential of the step's start
        if (parts) particle_substeps(c, phi.data(), pos, vel, dt, acc);
        // (b) full drift: kinetic phase in Fourier space
        drift(c, psi, dt);
        // (c) potential of the wave density plus the deposited baryons
        total_potential(c, psi, pos, phi.data());
        add_external(c, phi_ext, phi.data());
        // (d) second half kick with the new potential
        kick(c, psi, phi.data(), 0.5 * dt);
        if (parts) particle_kick(c, phi.data(), pos, vel, 0.5 * dt / S, acc);
        // absorbing boundary (Algorithm 1, after step (d))
        if (!mask.empty())
            for (int64_t i = 0; i < n; ++i) psi[i] *= mask[size_t(i)];
    }
}

}  // namespace orc

using namespace orc;

extern "C" {

void orc_poisson(const orc_config* c, const double* rho, double* phi) { poisson(c, rho, phi); }

void orc_cic_deposit(const orc_config* c, const double* pos, double* rho_b) {
    cic_deposit(c, pos, rho_b);
}

void orc_cic_force(const orc_config* c, const double* phi, const double* pos, double* acc) {
    cic_force(c, phi, pos, acc);
}

void orc_potential(const orc_config* c, const double* psi, const double* pos, double* phi) {
    total_potential(c, reinterpret_cast<const cplx*>(psi), pos, phi);
}

void orc_kdk(const orc_config* c, double* psi, double* pos, double* vel, int64_t nsteps,
             double dt) {
    kdk(c, reinterpret_cast<cplx*>(psi), pos, vel, nsteps, dt, nullptr);
}

void orc_kdk_ext(const orc_config* c, double* psi, double* pos, double* vel, int64_t nsteps,
                 double dt, const double* phi_ext) {
    kdk(c, reinterpret_cast<cplx*>(psi), pos, vel, nsteps, dt, phi_ext);
}

void orc_poisson_direct(const orc_config* c, const double* rho, double* phi) {
    Grid g(c);
    const double self = cube_self_integral();
    for (int64_t i = 0; i < g.nx; ++i)
        for (int64_t j = 0; j < g.ny; ++j)
            for (int64_t k = 0; k < g.nz; ++k) {
                double sum = 0.0;
                for (int64_t a = 0; a < g.nx; ++a)
                    for (int64_t b = 0; b < g.ny; ++b)
                        for (int64_t d = 0; d < g.nz; ++d)
                            sum += green_iso(c, g, i - a, j - b, k - d, self) *
                                   rho[(a * g.ny + b) * g.nz + d];
                phi[(i * g.ny + j) * g.nz + k] = sum;
            }
}

// The same direct sum evaluated at listed nodes only (i, j, k triples), so that
// the potential of a large grid can be checked node by node.
void orc_poisson_direct_at(const orc_config* c, const double* rho, const int64_t* nodes,
                           int64_t count, double* phi) {
    Grid g(c);
    const double self = cube_self_integral();
    for (int64_t n = 0; n < count; ++n) {
        const int64_t i = nodes[3 * n], j = nodes[3 * n + 1], k = nodes[3 * n + 2];
        double sum = 0.0;
        for (int64_t a = 0; a < g.nx; ++a)
            for (int64_t b = 0; b < g.ny; ++b)
                for (int64_t d = 0; d < g.nz; ++d)
                    sum += green_iso(c, g, i - a, j - b, k - d, self) *
                           rho[(a * g.ny + b) * g.nz + d];
        phi[n] = sum;
    }
}

double orc_cube_self_integral(void) { return cube_self_integral(); }

// Tidal potential with its mean acceleration removed (Sec. 4.3): the mean
// gradient along each axis over the nodes symmetric about the centre node
// (1 .. n-1; node 0 has no mirror in a periodic box of even n), averaged over
// the other two axes, is subtracted as a linear ramp through the box centre.
void orc_tidal_correct(const orc_config* c, const double* in, double* out) {
    Grid g(c);
    const int64_t n[3] = {g.nx, g.ny, g.nz};
    const double h[3] = {g.dx, g.dy, g.dz}, L[3] = {g.lx, g.ly, g.lz};
    double grad[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < g.nx; ++i)
        for (int64_t j = 0; j < g.ny; ++j)
            for (int64_t k = 0; k < g.nz; ++k) {
                const int64_t idx[3] = {i, j, k};
                for (int a = 0; a < 3; ++a) {
                    if (idx[a] != n[a] - 1) continue;
                    int64_t lo[3] = {i, j, k};
                    lo[a] = 1;
                    const double d = in[(i * g.ny + j) * g.nz + k] -
                                     in[(lo[0] * g.ny + lo[1]) * g.nz + lo[2]];
                    grad[a] += d / (double(n[a] - 2) * h[a]);
                }
            }
    for (int a = 0; a < 3; ++a) grad[a] /= double(g.n() / n[a]);
    for (int64_t i = 0; i < g.nx; ++i)
        for (int64_t j = 0; j < g.ny; ++j)
            for (int64_t k = 0; k < g.nz; ++k) {
                const double x[3] = {i * h[0] - 0.5 * L[0], j * h[1] - 0.5 * L[1],
                                     k * h[2] - 0.5 * L[2]};
                const int64_t o = (i * g.ny + j) * g.nz + k;
                out[o] = in[o] - grad[0] * x[0] - grad[1] * x[1] - grad[2] * x[2];
            }
}

void orc_energy_ext(const orc_config* c, const double* psi_in, const double* pos,
                    const double* vel, const double* phi_ext, double* out) {
    Grid g(c);
    const cplx* psi = reinterpret_cast<const cplx*>(psi_in);
    const int64_t n = g.n();
    std::vector<double> phi(n), rho(n, 0.0);
    if (c->n_particles > 0) cic_deposit(c, pos, rho.data());
    double mass = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double d = std::norm(psi[i]);
        mass += d;
        rho[i] += d;
    }
    poisson(c, rho.data(), phi.data());
    std::vector<cplx> f(psi, psi + n);
    fft3d(f.data(), int(g.nx), int(g.ny), int(g.nz), -1);
    double ek = 0.0;
    for (int64_t i = 0; i < g.nx; ++i)
        for (int64_t j = 0; j < g.ny; ++j)
            for (int64_t k = 0; k < g.nz; ++k)
                ek += g.k2(i, j, k) * std::norm(f[(i * g.ny + j) * g.nz + k]);
    const double eta = c->hbar_over_m;
    ek *= 0.5 * eta * eta * g.dv / double(n);
    // an external potential enters once (not halved) and is part of the
    // potential the wave feels
    double ep = 0.0, maxphi = 0.0, rho4 = 0.0, maxrho = 0.0, ex = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        ep += rho[i] * phi[i];
        const double pe = phi_ext ? phi_ext[i] : 0.0;
        ex += rho[i] * pe;
        maxphi = std::max(maxphi, std::fabs(phi[i] + pe));
        const double d = std::norm(psi[i]);
        rho4 += d * d;
        maxrho = std::max(maxrho, d);
    }
    ep *= 0.5 * g.dv;
    const double es = 0.5 * c->kappa * rho4 * g.dv;
    double kp = 0.0, mom[3] = {0.0, 0.0, 0.0};
    for (int64_t p = 0; p < c->n_particles; ++p)
        for (int a = 0; a < 3; ++a) {
            const double v = vel[3 * p + a];
            kp += v * v;
            mom[a] += v;
        }
    kp *= 0.5 * c->particle_mass;
    out[0] = mass * g.dv;
    out[1] = ek;
    out[2] = ep;
    out[3] = kp;
    ex *= g.dv;
    out[4] = ek + ep + kp + es + ex;
    for (int a = 0; a < 3; ++a) out[5 + a] = mom[a] * c->particle_mass;
    out[8] = maxphi;
    out[9] = es;
    out[10] = maxrho;
    out[11] = ex;
}

void orc_energy(const orc_config* c, const double* psi_in, const double* pos, const double* vel,
                double* out) {
    orc_energy_ext(c, psi_in, pos, vel, nullptr, out);
}

void orc_paper_energies(const orc_config* c, const double* psi_in, const double* phi, double* out) {
    Grid g(c);
    const cplx* psi = reinterpret_cast<const cplx*>(psi_in);
    const double h[3] = {g.dx, g.dy, g.dz};
    const double eta = c->hbar_over_m;
    double K = 0.0, Q = 0.0, V = 0.0, P[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < g.nx; ++i)
        for (int64_t j = 0; j < g.ny; ++j)
            for (int64_t k = 0; k < g.nz; ++k) {
                const int64_t o = g.at(i, j, k);
                const double rho = std::norm(psi[o]);
                int64_t nb[3][2] = {{g.at(i + 1, j, k), g.at(i - 1, j, k)},
                                    {g.at(i, j + 1, k), g.at(i, j - 1, k)},
                                    {g.at(i, j, k + 1), g.at(i, j, k - 1)}};
                double j2 = 0.0, q2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    // momentum density rho v = eta Im(psi* grad psi)
                    const cplx dpsi = (psi[nb[a][0]] - psi[nb[a][1]]) / (2.0 * h[a]);
                    const double ja = eta * (std::conj(psi[o]) * dpsi).imag();
                    j2 += ja * ja;
                    P[a] += ja;
                    const double ds = (std::sqrt(std::norm(psi[nb[a][0]])) -
                                       std::sqrt(std::norm(psi[nb[a][1]]))) / (2.0 * h[a]);
                    q2 += ds * ds;
                }
                if (rho > 1e-30) K += 0.5 * j2 / rho;
                Q += q2;
                V += rho * phi[o];
            }
    out[0] = K * g.dv;
    out[1] = Q * g.dv;
    out[2] = V * g.dv;
    out[3] = 2.0 * out[0] + 2.0 * out[1] + out[2];
    for (int a = 0; a < 3; ++a) out[4 + a] = P[a] * g.dv;
}

// Radii enclosing the fractions f of the wave mass around the node `centre`
// (App. A.1.2, spherical symmetry assumed).  Distances are minimum-image node
// distances r = dx sqrt(s), s = di^2 + dj^2 + dk^2 an integer (cubic cells);
// r_f is the smallest node distance whose enclosed mass (all nodes at that
// distance or closer) reaches f times the total.
int orc_mass_fraction_radii(const orc_config* c, const double* psi_in, const int32_t* centre,
                            const double* fractions, int nf, double* radii) {
    Grid g(c);
    if (!(g.dx == g.dy && g.dy == g.dz)) return -1;
    const cplx* psi = reinterpret_cast<const cplx*>(psi_in);
    const int64_t smax = (g.nx / 2) * (g.nx / 2) + (g.ny / 2) * (g.ny / 2) + (g.nz / 2) * (g.nz / 2);
    std::vector<double> shell(size_t(smax + 1), 0.0);
    auto offset = [](int64_t i, int64_t ci, int64_t n) {
        int64_t d = ((i - ci) % n + n) % n;   // in [0, n)
        return d >= n / 2 ? n - d : d;        // minimum image |offset|
    };
    double total = 0.0;
    for (int64_t i = 0; i < g.nx; ++i)
        for (int64_t j = 0; j < g.ny; ++j)
            for (int64_t k = 0; k < g.nz; ++k) {
                const int64_t di = offset(i, centre[0], g.nx), dj = offset(j, centre[1], g.ny),
                              dk = offset(k, centre[2], g.nz);
                const double m = std::norm(psi[g.at(i, j, k)]);
                shell[size_t(di * di + dj * dj + dk * dk)] += m;
                total += m;
            }
    for (int f = 0; f < nf; ++f) {
        double cum = 0.0;
        radii[f] = -1.0;
        for (int64_t s = 0; s <= smax; ++s) {
            cum += shell[size_t(s)];
            if (shell[size_t(s)] > 0.0 && cum >= fractions[f] * total) {
                radii[f] = g.dx * std::sqrt(double(s));
                break;
            }
        }
    }
    return 0;
}

double orc_dt_auto(const orc_config* c, const double* phi, const double* psi_in, double zeta,
                   double c_kin) {
    Grid g(c);
    double m = 0.0;
    for (int64_t i = 0; i < g.n(); ++i) m = std::max(m, std::fabs(phi[i]));
    const double h = std::min(g.dx, std::min(g.dy, g.dz));
    const double eta = c->hbar_over_m;
    double t = c_kin * h * h / eta;
    if (m > 0.0) t = std::min(t, kTwoPi * eta / m);
    if (c->kappa != 0.0 && psi_in) {
        const cplx* psi = reinterpret_cast<const cplx*>(psi_in);
        double r = 0.0;
        for (int64_t i = 0; i < g.n(); ++i) r = std::max(r, std::norm(psi[i]));
        if (r > 0.0) t = std::min(t, kTwoPi * eta / (std::fabs(c->kappa) * r));
    }
    return zeta * 0.5 * t;
}

void orc_absorb_mask(const orc_config* c, double dt, double* mask) { absorb_mask(c, dt, mask); }

}  // extern "C"
