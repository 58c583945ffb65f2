// Host side of libwdm: plan creation (workspace carving, FP64 twiddles),
// the merged kick-drift-kick schedule of Algorithm 1, diagnostics, profiling
// and the C ABI declared in include/wdm.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "wdm.h"
#include "wdm_internal.hpp"

namespace wdm {
// corrector (corrector.hip)
hipError_t conv_forward_layer(hipStream_t s, int layer, const uint16_t* in, const uint16_t* w,
                              const float* b, void* out, int n);
hipError_t conv_backward_data(hipStream_t s, int layer, const uint16_t* dz, const uint16_t* wbwd,
                              const uint16_t* act_in, uint16_t* dact, int n);
hipError_t conv_backward_weight(hipStream_t s, int layer, const uint16_t* dz,
                                const uint16_t* act_in, float* part, int nblocks, float* out,
                                int n);
int wgrad_row(int layer);
hipError_t net_pack_input(hipStream_t s, const float* x, uint16_t* y, int64_t cells, int cin,
                          int cp, const double* scales);
hipError_t net_mse(hipStream_t s, const float* y, const float* t, uint16_t* dy, double* part,
                   double* out, int64_t cells, int cout, int cp, const double* s_out);
hipError_t net_adam(hipStream_t s, float* w, const float* g, float* m, float* v, int n, float lr,
                    float b1, float b2, float eps, float c1, float c2);
hipError_t net_pack_weights(hipStream_t s, const float* w, uint16_t* fwd, uint16_t* bwd, int cin,
                            int cout, int cpin, int cpout);
hipError_t net_state_pack(hipStream_t s, const float* psi, const float* phi, uint16_t* x0,
                          int64_t cells, double* scal, double* part);
// the network's last layer with psi += s_out d fused into its epilogue and the
// FP64 mass of the corrected psi; with `rescale`, psi *= sqrt(mass before /
// mass after) (else the Poisson rebuild's density pass applies it)
hipError_t net_last_layer_apply(hipStream_t s, const uint16_t* in, const uint16_t* w,
                                const float* b, float* psi, int n, double* scal, double* part,
                                bool rescale);
hipError_t net_pair(hipStream_t s, const float* psi, const float* phi, const float* target,
                    float* x, float* y, int64_t cells);
hipError_t net_moments(hipStream_t s, const float* x, const float* y, int64_t cells, double* rows,
                       bool first);
hipError_t net_fit_scales(hipStream_t s, const double* rows, double count, double* scal);
hipError_t net_set_scales(hipStream_t s, double* scal, double s_psi, double s_phi, double s_out);
size_t net_moment_doubles();
hipError_t net_unpack_grads(hipStream_t s, const float* sum, float* gw, float* gb, int cin,
                            int cout, int cpin, int row);
hipError_t launch_restrict_modes(hipStream_t s, const void* fine, void* coarse, int nf, int nc,
                                 int prec);
hipError_t launch_contrast(const Launch& L, int prec, int64_t n);
hipError_t launch_shells(const Launch& L, int prec, int nbins, double* part, double* out);
hipError_t launch_distance(const Launch& L, int prec, const void* other, int64_t n, double* part,
                           double* out);
size_t shells_partial_doubles();
int64_t axis_tiles(int n, int64_t pencils, int prec);
hipError_t launch_scale_complex(hipStream_t s, void* p, int64_t n, double scale, int prec);
int sort_blocks(int64_t np);
}  // namespace wdm

using namespace wdm;

namespace {

thread_local std::string g_err;

wdm_status fail(wdm_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

constexpr size_t kAlign = 256;
// kinetic constant of the CFL step (Sec. 3.5): dt_max = 0.5 min{(4 / (3 pi)) dx^2 / eta, ...}
constexpr double kCKin = 4.0 / (3.0 * kPi);
// merged steps per replayed step graph (runs of steps between re-sorts)
constexpr int kStepChunk = 8;
// resident particle work-groups per CU where the particle kernel is the longer
// branch of a step or runs alone (deposits of a state); the default (four)
// leaves room for the psi passes it overlaps
constexpr int kPartsAlone = 8;

struct Carver {
    size_t off = 0;
    size_t take(size_t bytes) {
        off = (off + kAlign - 1) / kAlign * kAlign;
        const size_t o = off;
        off += bytes;
        return o;
    }
};

struct MemberLayout {
    size_t psi, phi, rho_b, spec, nyq, kin, absorb, dt, results, watch, stab, rho_fx = 0;
    size_t pad = 0, green = 0, ext = 0;   // vacuum boundary, external potential
    size_t p[7], a[7], key_a, key_b, idx_a, idx_b, hist;
};

struct Layout {
    std::vector<MemberLayout> m;
    std::map<int, size_t> tw;     // axis length -> twiddle table offset
    size_t scratch = 0, partials = 0, table = 0, iso_table = 0, pk = 0, total = 0;
    int64_t partial_rows = 0;
};

enum Kind : int {
    kKZPot = 0, kKParticles, kKYPsiF, kKXKin, kKYPsiI, kKZDens, kKYSpecF, kKXGreen, kKYSpecI,
    kKClose, kKCloseParticles, kKSort, kKVacuum, kKPhiR2C, kKinds
};
const char* kKindNames[kKinds] = {"z_potential_kick", "particles_kick_drift_deposit",
                                  "y_fft_psi_fwd",    "x_kinetic",
                                  "y_fft_psi_inv",    "z_density_r2c",
                                  "y_fft_spec_fwd",   "x_green",
                                  "y_fft_spec_inv",   "z_potential_close_kick",
                                  "particles_close_kick", "particle_sort",
                                  "vacuum_poisson",   "z_phi_r2c"};

bool valid_config(const wdm_config& c, std::string& why) {
    if (!axis_supported(c.nx) || !axis_supported(c.ny) || !axis_supported(c.nz)) {
        why = "axis lengths must be in {16,32,64,96,128,192,256,384,512}";
        return false;
    }
    if (!(c.lx > 0 && c.ly > 0 && c.lz > 0)) {
        why = "box lengths must be positive";
        return false;
    }
    if (!(c.hbar_over_m > 0) || !std::isfinite(c.four_pi_G)) {
        why = "hbar_over_m must be positive and four_pi_G finite";
        return false;
    }
    if (c.n_particles < 0 || c.n_particles > (int64_t(1) << 31) - 1) {
        why = "n_particles out of range";
        return false;
    }
    if (c.n_particles > 0 && !(c.particle_mass >= 0 && std::isfinite(c.particle_mass))) {
        why = "particle_mass must be finite and non-negative";
        return false;
    }
    if (c.precision != WDM_C64 && c.precision != WDM_C128) {
        why = "precision must be WDM_C64 or WDM_C128";
        return false;
    }
    if ((c.flags & ~uint32_t(WDM_DETERMINISTIC_DEPOSIT | WDM_STRICT_CFL)) != 0) {
        why = "flags may only hold WDM_DETERMINISTIC_DEPOSIT and WDM_STRICT_CFL";
        return false;
    }
    if (!std::isfinite(c.kappa) || !std::isfinite(c.absorb_alpha) || c.absorb_alpha < 0) {
        why = "kappa must be finite and absorb_alpha finite and >= 0";
        return false;
    }
    if (c.absorb_alpha > 0 && !(c.absorb_nb > 0 && std::isfinite(c.absorb_nb))) {
        why = "absorb_nb must be positive when the absorbing boundary is on";
        return false;
    }
    if (c.baryon_mode != WDM_BARYON_DYNAMIC && c.baryon_mode != WDM_BARYON_STATIC) {
        why = "baryon_mode must be WDM_BARYON_DYNAMIC or WDM_BARYON_STATIC";
        return false;
    }
    if (c.nbody_substeps < 0 || c.nbody_substeps > 1024) {
        why = "nbody_substeps must be in [0, 1024]";
        return false;
    }
    if (c.boundary != WDM_BOUNDARY_PERIODIC && c.boundary != WDM_BOUNDARY_VACUUM) {
        why = "boundary must be WDM_BOUNDARY_PERIODIC or WDM_BOUNDARY_VACUUM";
        return false;
    }
    if (c.boundary == WDM_BOUNDARY_VACUUM) {
        const double h = c.lx / c.nx;
        if (h != c.ly / c.ny || h != c.lz / c.nz) {
            why = "the vacuum boundary needs cubic cells";
            return false;
        }
        if (!axis_supported(2 * c.nx) || !axis_supported(2 * c.ny) || !axis_supported(2 * c.nz)) {
            why = "the vacuum boundary needs axis lengths <= 256 (padded to 2n)";
            return false;
        }
    }
    if (c.external_potential != 0 && c.external_potential != 1) {
        why = "external_potential must be 0 or 1";
        return false;
    }
    return true;
}

bool make_layout(const wdm_config* mem, int n, Layout& L, std::string& why) {
    if (!mem || n <= 0) {
        why = "need at least one member";
        return false;
    }
    const int prec = mem[0].precision;
    for (int i = 0; i < n; ++i) {
        if (!valid_config(mem[i], why)) {
            why = "member " + std::to_string(i) + ": " + why;
            return false;
        }
        if (mem[i].precision != prec) {
            why = "all members must share one precision";
            return false;
        }
        if ((mem[i].flags ^ mem[0].flags) & WDM_DETERMINISTIC_DEPOSIT) {
            why = "all members must share the WDM_DETERMINISTIC_DEPOSIT flag";
            return false;
        }
    }
    const size_t cs = prec ? 16 : 8, rs = prec ? 8 : 4;
    Carver c;
    int64_t maxn = 0, maxplane = 0;
    L.m.resize(n);
    for (int i = 0; i < n; ++i) {
        const wdm_config& g = mem[i];
        const int64_t cells = int64_t(g.nx) * g.ny * g.nz;
        maxn = std::max(maxn, cells);
        maxplane = std::max(maxplane, int64_t(g.ny) * g.nz);
        MemberLayout& m = L.m[i];
        m.psi = c.take(cells * cs);
        m.phi = c.take(cells * rs);
        m.rho_b = c.take(cells * rs);
        m.spec = c.take(int64_t(g.nx) * g.ny * (g.nz / 2) * cs);
        m.nyq = c.take(int64_t(g.nx) * g.ny * cs);
        m.kin = c.take((int64_t(g.nx) + int64_t(g.ny) * g.nz) * 16);
        m.absorb = c.take((int64_t(g.nx) + g.ny + g.nz) * sizeof(double));
        if (g.boundary == WDM_BOUNDARY_VACUUM) {
            m.pad = c.take(8 * cells * cs);
            m.green = c.take((int64_t(g.nx) + 1) * (g.ny + 1) * (g.nz + 1) * rs);
        }
        if (g.external_potential) m.ext = c.take(cells * rs);
        m.dt = c.take(4 * sizeof(double));
        m.results = c.take(kRedFields * sizeof(double));
        m.watch = c.take(watch_words(g.nx, g.ny) * sizeof(unsigned long long));
        m.stab = c.take(2 * sizeof(double));
        if (g.flags & WDM_DETERMINISTIC_DEPOSIT) m.rho_fx = c.take(cells * 8);
        const int64_t np = std::max<int64_t>(g.n_particles, 0);
        for (int a = 0; a < 7; ++a) m.p[a] = c.take(np * 4);
        for (int a = 0; a < 7; ++a) m.a[a] = c.take(np * 4);
        m.key_a = c.take(np * 4);
        m.key_b = c.take(np * 4);
        m.idx_a = c.take(np * 4);
        m.idx_b = c.take(np * 4);
        m.hist = c.take(int64_t(256) * (std::max(1, sort_blocks(np)) + 1) * 4);
        for (int len : {g.nx, g.ny, g.nz})
            if (!L.tw.count(len)) L.tw[len] = 0;
        if (g.boundary == WDM_BOUNDARY_VACUUM)
            for (int len : {2 * g.nx, 2 * g.ny, 2 * g.nz})
                if (!L.tw.count(len)) L.tw[len] = 0;
    }
    // complex64: hi and lo float tables; complex128: one double table
    for (auto& kv : L.tw) kv.second = c.take(size_t(kv.first) * cs * (prec ? 1 : 2));
    L.scratch = c.take(maxn * cs);
    L.partial_rows = std::max<int64_t>(kRedBlocks, (maxplane + 7) / 8);
    L.partials = c.take(L.partial_rows * kRedFields * sizeof(double));
    L.table = c.take(n * sizeof(MemberDev));
    L.iso_table = c.take(n * sizeof(MemberDev));
    L.pk = c.take(shells_partial_doubles() * sizeof(double));
    L.total = (c.off + kAlign - 1) / kAlign * kAlign;
    return true;
}

// Step passes whose FFT plan the autotuner chooses (per size class).
enum TuneSlot : int { kTzPot = 0, kTyPsi, kTxKin, kTzDens, kTySpec, kTxGreen, kTuneSlots };

struct SizeClass {
    int first, count;       // device-table range
    int nx, ny, nz;
    int64_t max_np;
    int var[kTuneSlots] = {0, 0, 0, 0, 0, 0};   // plan variant per tunable pass
    bool absorb = false;    // some member has an absorbing boundary
    bool extended = false;  // some member has a self-interaction or absorbing boundary
    int64_t moving_np = 0;  // most particles of a member whose particles move
    bool vacuum = false;    // isolated Poisson solve (the class's members share the boundary)
};

struct Rec {
    int kind;
    hipEvent_t a, b;
};

}  // namespace

namespace wdm {
void set_last_error(const std::string& msg) { g_err = msg; }
}  // namespace wdm


struct wdm_plan {
    hipStream_t stream = nullptr;
    int prec = 0;
    std::vector<wdm_config> cfg;        // user order
    std::vector<int> dev_index;         // user member -> device table slot
    std::vector<MemberDev> host;        // device-table order
    std::vector<SizeClass> classes;
    std::vector<bool> has_state;        // user order
    MemberDev* table = nullptr;
    MemberDev* iso_table = nullptr;     // padded-grid descriptors of vacuum members
    std::vector<MemberDev> iso_host;
    Layout layout;
    uint8_t* ws = nullptr;
    int sort_interval = 32;
    int64_t steps_done = 0;
    bool det = false;                   // WDM_DETERMINISTIC_DEPOSIT (shared by all members)
    bool profiling = false;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    size_t pool_next = 0;
    // captured-step machinery: an internal stream pair joined to the caller's
    // stream by events; the particle kernel runs on a forked graph branch
    bool use_graphs = true;
    hipStream_t s_main = nullptr, s_aux = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_fork = nullptr, ev_join = nullptr;
    // [0] the opening half kick, [1] one merged step, [2] kStepChunk merged
    // steps (fewer graph launches: each launch boundary idles the device)
    hipGraphExec_t g_step[3] = {nullptr, nullptr, nullptr};
    // attached corrector (wdm_plan_attach_corrector): applied to member
    // net_member after every `every` steps; corr_phase counts the steps since
    // the last application.  g_block holds `every` steps, the closing half kick
    // and the correction as one captured graph.
    wdm_net* net = nullptr;
    int32_t net_member = 0;
    int32_t every = 0;
    int64_t corr_phase = 0;
    hipGraphExec_t g_block = nullptr;
};

namespace {

hipEvent_t take_event(wdm_plan* p) {
    if (p->pool_next == p->pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        p->pool.push_back(e);
    }
    return p->pool[p->pool_next++];
}

// Bracket one launch with HIP events on the stream it is launched on.
template <class F>
hipError_t timed_on(wdm_plan* p, hipStream_t s, int kind, F&& f) {
    if (!p->profiling) return f();
    hipEvent_t a = take_event(p), b = take_event(p);
    if (!a || !b) return f();
    if (const hipError_t r = hipEventRecord(a, s); r != hipSuccess) return r;
    const hipError_t e = f();
    if (const hipError_t r = hipEventRecord(b, s); r != hipSuccess) return r;
    p->recs.push_back({kind, a, b});
    return e;
}
template <class F>
hipError_t timed(wdm_plan* p, int kind, F&& f) {
    return timed_on(p, p->stream, kind, f);
}

#define HIPCHK(expr)                                                                  \
    do {                                                                              \
        const hipError_t e_ = (expr);                                                 \
        if (e_ != hipSuccess)                                                         \
            return fail(WDM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

int64_t cells_of(const wdm_config& c) { return int64_t(c.nx) * c.ny * c.nz; }

wdm_status check_member(wdm_plan* p, int32_t member) {
    if (!p) return fail(WDM_EINVAL, "null plan");
    if (member < 0 || member >= int32_t(p->cfg.size()))
        return fail(WDM_EINVAL, "member index out of range");
    return WDM_OK;
}

Launch one(wdm_plan* p, int32_t member) {
    return Launch{p->stream, p->table, p->dev_index[member], 1};
}

// Vacuum-boundary Poisson solve of a class (or one member): the density,
// computed by P5 (`op`: from psi after its inverse z transform, or from psi in
// real space) into Phi, is convolved with the free-space Green's function on
// the zero-padded grid, and the potential is handed to the next P1 as the half
// spectrum along z, as the periodic solve does.
hipError_t enqueue_vacuum_poisson(wdm_plan* p, hipStream_t s, int first, int count, int nx,
                                  int ny, int nz, DensOp op) {
    const int prec = p->prec;
    const Launch L{s, p->table, first, count};
    const Launch LP{s, p->iso_table, first, count};
    hipError_t e = timed_on(p, s, kKZDens,
                            [&] { return launch_z_density(L, prec, nx, ny, nz, op); });
    if (e != hipSuccess) return e;
    // The padded density is zero outside the x < nx, y < ny corner: the forward
    // z pass reads the density rows and fills only those padded rows, the y
    // passes treat the y >= ny half of each x < nx pencil as zeros (forward) or
    // leave it unstored (inverse), the x pass reads and writes the x < nx half
    // with the other half implied zero, and the inverse z pass writes the
    // corner's real part to Phi.  No other part of the padded grid is read.
    e = timed_on(p, s, kKVacuum, [&] {
        const int px = 2 * nx, py = 2 * ny, pz = 2 * nz;
        hipError_t r = launch_vac_fft(LP, prec, px, py, pz, 0);
        if (r == hipSuccess) r = launch_vac_fft(LP, prec, px, py, pz, 1);
        if (r == hipSuccess) r = launch_x_mul_green(LP, prec, px, py, pz);
        if (r == hipSuccess) r = launch_vac_fft(LP, prec, px, py, pz, 2);
        if (r == hipSuccess) r = launch_vac_fft(LP, prec, px, py, pz, 3);
        return r;
    });
    if (e != hipSuccess) return e;
    return timed_on(p, s, kKPhiR2C,
                    [&] { return launch_z_density(L, prec, nx, ny, nz, kPhiR2C); });
}

// Transform of the padded Green's function of every vacuum class (once per plan).
hipError_t compute_green(wdm_plan* p) {
    hipError_t e = hipSuccess;
    for (const auto& c : p->classes) {
        if (!c.vacuum) continue;
        const Launch L{p->stream, p->table, c.first, c.count};
        const Launch LP{p->stream, p->iso_table, c.first, c.count};
        const int64_t cells = int64_t(c.nx) * c.ny * c.nz;
        if ((e = launch_green_fill(L, p->prec, cells)) != hipSuccess) return e;
        for (int axis = 2; axis >= 0; --axis)
            if ((e = launch_axis_fft(LP, p->prec, 2 * c.nx, 2 * c.ny, 2 * c.nz, axis, false, 0)) !=
                hipSuccess)
                return e;
        if ((e = launch_green_extract(L, p->prec, cells)) != hipSuccess) return e;
    }
    return e;
}

// A member's extended kick (self-interaction, absorbing boundary, external
// potential) as its class launches it.
bool member_extended(const wdm_config& c) {
    return c.kappa != 0.0 || c.absorb_alpha != 0.0 || c.external_potential != 0;
}

// Poisson solve of the density already deposited in rho_b plus |psi|^2
// (psi in real space), ending with Phi written and psi untouched.
hipError_t potential_from_state(wdm_plan* p, const Launch& L, const wdm_config& c,
                                const double* rescale = nullptr) {
    hipError_t e;
    if (c.boundary == WDM_BOUNDARY_VACUUM) {
        if (rescale != nullptr) return hipErrorInvalidValue;
        e = enqueue_vacuum_poisson(p, L.stream, L.first, L.count, c.nx, c.ny, c.nz,
                                   kDensDirectToPhi);
        if (e != hipSuccess) return e;
    } else {
        if ((e = launch_z_density(L, p->prec, c.nx, c.ny, c.nz, kDensDirect, 0, -1, rescale)) !=
            hipSuccess)
            return e;
        if ((e = launch_y_fft_spec(L, p->prec, c.nx, c.ny, c.nz, false)) != hipSuccess) return e;
        if ((e = launch_x_green(L, p->prec, c.nx, c.ny, c.nz)) != hipSuccess) return e;
        if ((e = launch_y_fft_spec(L, p->prec, c.nx, c.ny, c.nz, true)) != hipSuccess) return e;
    }
    return launch_z_potential_kick(L, p->prec, c.nx, c.ny, c.nz, kZPhiOnly, kHalfKick, 0,
                                   member_extended(c));
}

// Outcome of the stability checks of the steps since wdm_set_state (stab as
// read back from the device): a non-finite potential or density always fails,
// a step above dt_max only under WDM_STRICT_CFL.
wdm_status stability_status(const wdm_config& c, const double stab[2]) {
    if (stab[1] != 0.0) return fail(WDM_EUNSTABLE, "non-finite potential or density in a step");
    if ((c.flags & WDM_STRICT_CFL) && stab[0] > 1.0) {
        char msg[160];
        std::snprintf(msg, sizeof(msg),
                      "time step above the CFL bound of Sec. 3.5: |dt| / dt_max = %.6g", stab[0]);
        return fail(WDM_EUNSTABLE, msg);
    }
    return WDM_OK;
}

// The stability checks of a member's steps so far (synchronises the stream).
wdm_status check_stability(wdm_plan* p, int32_t member) {
    double stab[2];
    const MemberDev& m = p->host[p->dev_index[member]];
    HIPCHK(hipMemcpyAsync(stab, m.stab, sizeof(stab), hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    return stability_status(p->cfg[member], stab);
}

// Potential of a member's synchronised state (psi, particle positions): the
// moving particles are deposited (static ones keep their deposit in rho_b)
// and Poisson is solved, as wdm_set_state does.  `rho_b_ready`: rho_b already
// holds the deposit of the current positions (kept by the last step's P5), so
// it is not deposited again.  `rescale`: see launch_z_density (periodic only).
hipError_t rebuild_potential(wdm_plan* p, int32_t member, hipStream_t s, bool rho_b_ready = false,
                             const double* rescale = nullptr) {
    const wdm_config& c = p->cfg[member];
    const Launch L{s, p->table, p->dev_index[member], 1};
    if (!rho_b_ready && c.n_particles > 0 && c.baryon_mode == WDM_BARYON_DYNAMIC) {
        const hipError_t e =
            launch_particles(L, p->prec, c.n_particles, 2, kHalfKick, p->det, kPartsAlone);
        if (e != hipSuccess) return e;
    }
    return potential_from_state(p, L, c, rescale);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* wdm_last_error(void) { return g_err.c_str(); }

size_t wdm_workspace_bytes(const wdm_config* members, int32_t n_members) {
    Layout L;
    std::string why;
    if (!make_layout(members, n_members, L, why)) {
        g_err = why;
        return 0;
    }
    return L.total;
}

wdm_status wdm_plan_create(const wdm_config* members, int32_t n_members, void* workspace,
                           size_t workspace_bytes, void* hip_stream, wdm_plan** out) {
    if (!out) return fail(WDM_EINVAL, "out is null");
    *out = nullptr;
    Layout L;
    std::string why;
    if (!make_layout(members, n_members, L, why)) return fail(WDM_EINVAL, why);
    if (!workspace) return fail(WDM_EINVAL, "workspace is null");
    if (workspace_bytes < L.total)
        return fail(WDM_ENOMEM, "workspace of " + std::to_string(workspace_bytes) +
                                    " bytes < required " + std::to_string(L.total));
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
        return fail(WDM_EINVAL, "workspace must be 256-byte aligned");
    auto* p = new wdm_plan();
    p->stream = static_cast<hipStream_t>(hip_stream);
    p->prec = members[0].precision;
    p->cfg.assign(members, members + n_members);
    p->layout = L;
    p->ws = static_cast<uint8_t*>(workspace);
    p->has_state.assign(n_members, false);
    p->det = (members[0].flags & WDM_DETERMINISTIC_DEPOSIT) != 0;
    uint8_t* ws = p->ws;
    const size_t cs = p->prec ? 16 : 8;

    // group members into size classes (identical grids), contiguous in the table
    std::vector<int> order(n_members);
    for (int i = 0; i < n_members; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const auto& A = members[a];
        const auto& B = members[b];
        return std::make_tuple(A.boundary, A.nx, A.ny, A.nz) <
               std::make_tuple(B.boundary, B.nx, B.ny, B.nz);
    });
    p->dev_index.assign(n_members, 0);
    p->host.resize(n_members);
    p->iso_host.resize(n_members);
    for (int d = 0; d < n_members; ++d) {
        const int u = order[d];
        p->dev_index[u] = d;
        const wdm_config& c = members[u];
        const MemberLayout& ml = L.m[u];
        MemberDev& m = p->host[d];
        std::memset(&m, 0, sizeof(m));
        m.psi = ws + ml.psi;
        m.phi = ws + ml.phi;
        m.rho_b = ws + ml.rho_b;
        m.spec = ws + ml.spec;
        m.spec_nyq = ws + ml.nyq;
        m.scratch = ws + L.scratch;
        m.kin = ws + ml.kin;
        m.absorb = reinterpret_cast<double*>(ws + ml.absorb);
        m.pad = c.boundary == WDM_BOUNDARY_VACUUM ? ws + ml.pad : nullptr;
        m.green = c.boundary == WDM_BOUNDARY_VACUUM ? ws + ml.green : nullptr;
        m.ext = c.external_potential ? ws + ml.ext : nullptr;
        m.tw_x = ws + L.tw.at(c.nx);
        m.tw_y = ws + L.tw.at(c.ny);
        m.tw_z = ws + L.tw.at(c.nz);
        m.nx = c.nx;
        m.ny = c.ny;
        m.nz = c.nz;
        m.lx = c.lx;
        m.ly = c.ly;
        m.lz = c.lz;
        m.eta = c.hbar_over_m;
        m.four_pi_G = c.four_pi_G;
        m.kappa = c.kappa;
        m.absorb_alpha = c.absorb_alpha;
        m.absorb_nb = c.absorb_nb;
        m.substeps = std::max(1, c.nbody_substeps);
        m.static_baryons = c.baryon_mode == WDM_BARYON_STATIC ? 1 : 0;
        m.inv_dx = double(c.nx) / c.lx;
        m.inv_dy = double(c.ny) / c.ly;
        m.inv_dz = double(c.nz) / c.lz;
        m.inv_lx = 1.0 / c.lx;
        m.inv_ly = 1.0 / c.ly;
        m.inv_lz = 1.0 / c.lz;
        m.dt = reinterpret_cast<double*>(ws + ml.dt);
        m.np = c.n_particles;
        float** pp[6] = {&m.px, &m.py, &m.pz, &m.vx, &m.vy, &m.vz};
        float** aa[6] = {&m.apx, &m.apy, &m.apz, &m.avx, &m.avy, &m.avz};
        for (int a = 0; a < 6; ++a) {
            *pp[a] = reinterpret_cast<float*>(ws + ml.p[a]);
            *aa[a] = reinterpret_cast<float*>(ws + ml.a[a]);
        }
        m.id = reinterpret_cast<int32_t*>(ws + ml.p[6]);
        m.aid = reinterpret_cast<int32_t*>(ws + ml.a[6]);
        m.key_a = reinterpret_cast<uint32_t*>(ws + ml.key_a);
        m.key_b = reinterpret_cast<uint32_t*>(ws + ml.key_b);
        m.idx_a = reinterpret_cast<uint32_t*>(ws + ml.idx_a);
        m.idx_b = reinterpret_cast<uint32_t*>(ws + ml.idx_b);
        m.hist = reinterpret_cast<uint32_t*>(ws + ml.hist);
        m.particle_mass = c.particle_mass;
        m.partials = reinterpret_cast<double*>(ws + L.partials);
        m.results = reinterpret_cast<double*>(ws + ml.results);
        m.watch = reinterpret_cast<unsigned long long*>(ws + ml.watch);
        m.watch_n = watch_slots(c.nx, c.ny);
        m.stab = reinterpret_cast<double*>(ws + ml.stab);
        if (c.flags & WDM_DETERMINISTIC_DEPOSIT) {
            // fixed point with round(value * 2^S): the largest possible node sum,
            // all the member's particle mass on one node, stays below 2^62
            m.deterministic = 1;
            m.rho_fx = reinterpret_cast<unsigned long long*>(ws + ml.rho_fx);
            const double total = double(c.n_particles) * c.particle_mass * m.inv_dx * m.inv_dy *
                                 m.inv_dz;
            int ex = 0;
            (void)std::frexp(total, &ex);
            m.fx_scale = std::ldexp(1.0, 62 - ex);
            m.fx_inv = std::ldexp(1.0, ex - 62);
        }
        if (p->classes.empty() || p->classes.back().nx != c.nx || p->classes.back().ny != c.ny ||
            p->classes.back().nz != c.nz ||
            p->classes.back().vacuum != (c.boundary == WDM_BOUNDARY_VACUUM)) {
            p->classes.push_back({d, 0, c.nx, c.ny, c.nz, 0});
            p->classes.back().vacuum = c.boundary == WDM_BOUNDARY_VACUUM;
        }
        p->classes.back().count++;
        p->classes.back().max_np = std::max<int64_t>(p->classes.back().max_np, c.n_particles);
        if (c.absorb_alpha != 0.0) p->classes.back().absorb = true;
        if (c.absorb_alpha != 0.0 || c.kappa != 0.0 || c.external_potential)
            p->classes.back().extended = true;
        if (c.baryon_mode == WDM_BARYON_DYNAMIC)
            p->classes.back().moving_np =
                std::max<int64_t>(p->classes.back().moving_np, c.n_particles);
    }
    p->table = reinterpret_cast<MemberDev*>(ws + L.table);
    p->iso_table = reinterpret_cast<MemberDev*>(ws + L.iso_table);
    // the padded grid of a vacuum member as a member of its own, for the plain
    // axis transforms: doubled lengths, its twiddles, the padded buffer as psi
    for (int d = 0; d < n_members; ++d) {
        const MemberDev& m = p->host[d];
        MemberDev& iso = p->iso_host[d];
        iso = m;
        if (!m.pad) continue;
        iso.nx = 2 * m.nx;
        iso.ny = 2 * m.ny;
        iso.nz = 2 * m.nz;
        iso.psi = m.pad;
        iso.scratch = m.pad;
        iso.tw_x = ws + L.tw.at(iso.nx);
        iso.tw_y = ws + L.tw.at(iso.ny);
        iso.tw_z = ws + L.tw.at(iso.nz);
    }

    auto cleanup = [&](wdm_status st, const std::string& msg) {
        delete p;
        return fail(st, msg);
    };
    // twiddles W_n^m = exp(-2 pi i m / n) in FP64; complex64 stores the
    // double-float split hi = float(w), lo = float(w - hi)
    for (const auto& kv : L.tw) {
        const int n = kv.first;
        std::vector<double> d(2 * size_t(n));
        std::vector<float> f(4 * size_t(n));
        for (int m = 0; m < n; ++m) {
            const double a = -kTwoPi * double(m) / double(n);
            d[2 * m] = std::cos(a);
            d[2 * m + 1] = std::sin(a);
            f[2 * m] = float(d[2 * m]);
            f[2 * m + 1] = float(d[2 * m + 1]);
            f[2 * n + 2 * m] = float(d[2 * m] - double(f[2 * m]));
            f[2 * n + 2 * m + 1] = float(d[2 * m + 1] - double(f[2 * m + 1]));
        }
        const void* src = p->prec ? static_cast<const void*>(d.data()) : f.data();
        const size_t bytes = size_t(n) * cs * (p->prec ? 1 : 2);
        if (const hipError_t e = hipMemcpy(ws + kv.second, src, bytes, hipMemcpyHostToDevice);
            e != hipSuccess)
            return cleanup(WDM_EDEVICE, std::string("twiddle upload failed: ") +
                                            hipGetErrorString(e));
    }
    if (hipMemcpy(p->table, p->host.data(), sizeof(MemberDev) * n_members,
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->iso_table, p->iso_host.data(), sizeof(MemberDev) * n_members,
                  hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(WDM_EDEVICE, "member table upload failed");
    // clear accumulators and slots that must start at zero
    for (int d = 0; d < n_members; ++d) {
        const MemberDev& m = p->host[d];
        const int64_t cells = int64_t(m.nx) * m.ny * m.nz;
        if (launch_zero(p->stream, m.rho_b, size_t(cells) * (p->prec ? 8 : 4)) != hipSuccess ||
            launch_zero(p->stream, m.dt, 4 * sizeof(double)) != hipSuccess ||
            launch_zero(p->stream, m.results, kRedFields * sizeof(double)) != hipSuccess ||
            launch_zero(p->stream, m.watch, (2 * m.watch_n + 2) * sizeof(unsigned long long)) !=
                hipSuccess ||
            launch_zero(p->stream, m.stab, 2 * sizeof(double)) != hipSuccess ||
            (m.rho_fx && launch_zero(p->stream, m.rho_fx, size_t(cells) * 8) != hipSuccess))
            return cleanup(WDM_EDEVICE, "plan initialisation failed");
    }
    // absorbing factors of dt = 0 (all ones) until the first step sets dt
    for (const auto& c : p->classes)
        if (launch_absorb_tables(Launch{p->stream, p->table, c.first, c.count}) != hipSuccess)
            return cleanup(WDM_EDEVICE, "plan initialisation failed");
    // no external potential until one is set
    for (int d = 0; d < n_members; ++d) {
        const MemberDev& m = p->host[d];
        if (m.ext && launch_zero(p->stream, m.ext, size_t(int64_t(m.nx) * m.ny * m.nz) *
                                                       (p->prec ? 8 : 4)) != hipSuccess)
            return cleanup(WDM_EDEVICE, "plan initialisation failed");
    }
    if (compute_green(p) != hipSuccess)
        return cleanup(WDM_EDEVICE, "Green's function of the vacuum boundary failed");
    if (hipStreamSynchronize(p->stream) != hipSuccess)
        return cleanup(WDM_EDEVICE, "plan initialisation failed");
    *out = p;
    g_err.clear();
    return WDM_OK;
}

wdm_status wdm_plan_destroy(wdm_plan* plan) {
    if (!plan) return fail(WDM_EINVAL, "null plan");
    (void)hipStreamSynchronize(plan->stream);
    if (plan->s_main) (void)hipStreamSynchronize(plan->s_main);
    if (plan->s_aux) (void)hipStreamSynchronize(plan->s_aux);
    for (hipEvent_t e : plan->pool) (void)hipEventDestroy(e);
    for (hipGraphExec_t g : plan->g_step)
        if (g) (void)hipGraphExecDestroy(g);
    if (plan->g_block) (void)hipGraphExecDestroy(plan->g_block);
    for (hipEvent_t e : {plan->ev_in, plan->ev_out, plan->ev_fork, plan->ev_join})
        if (e) (void)hipEventDestroy(e);
    if (plan->s_main) (void)hipStreamDestroy(plan->s_main);
    if (plan->s_aux) (void)hipStreamDestroy(plan->s_aux);
    delete plan;
    return WDM_OK;
}

wdm_status wdm_set_state(wdm_plan* p, int32_t member, const void* psi, const float* pos,
                         const float* vel, double t0) {
    if (wdm_status s = check_member(p, member)) return s;
    const wdm_config& c = p->cfg[member];
    if (!psi) return fail(WDM_EINVAL, "psi is null");
    if (c.n_particles > 0 && (!pos || !vel)) return fail(WDM_EINVAL, "pos/vel are null");
    if (!std::isfinite(t0)) return fail(WDM_EINVAL, "t0 must be finite");
    const Launch L = one(p, member);
    const MemberDev& m = p->host[p->dev_index[member]];
    const int64_t n = cells_of(c);
    HIPCHK(hipMemcpyAsync(m.psi, psi, size_t(n) * (p->prec ? 16 : 8), hipMemcpyDeviceToDevice,
                          p->stream));
    HIPCHK(launch_zero(p->stream, m.rho_b, size_t(n) * (p->prec ? 8 : 4)));
    HIPCHK(launch_zero(p->stream, m.watch, (2 * m.watch_n + 2) * sizeof(unsigned long long)));
    HIPCHK(launch_zero(p->stream, m.stab, 2 * sizeof(double)));
    if (c.n_particles > 0) {
        HIPCHK(launch_particle_upload(p->stream, m, pos, vel));
        HIPCHK(launch_particle_sort(L, c.n_particles, c.nx, c.ny, c.nz));
        HIPCHK(launch_particles(L, p->prec, c.n_particles, 2, kHalfKick, p->det, kPartsAlone));
    }
    HIPCHK(potential_from_state(p, L, c));
    HIPCHK(launch_reduce_grid(L, p->prec, n, 0));
    HIPCHK(launch_reduce_finish(L, 7, kRedBlocks, true));
    HIPCHK(launch_reduce_finish(L, 8, kRedBlocks, true));
    HIPCHK(launch_dt_auto(L, 0.9, kCKin));
    HIPCHK(launch_set_dt(L, t0, 3));
    p->has_state[member] = true;
    return WDM_OK;
}

wdm_status wdm_set_member_dt(wdm_plan* p, int32_t member, double dt) {
    if (wdm_status s = check_member(p, member)) return s;
    if (!std::isfinite(dt)) return fail(WDM_EINVAL, "dt must be finite");
    HIPCHK(launch_set_dt(one(p, member), dt, 2));
    return WDM_OK;
}

}  // extern "C"

namespace {

// One merged KDK step for every size class (P1, particles, P2 ... P8).  With
// `aux` set the particle kernel is forked onto it after P1 and joined before
// P5, so it overlaps the y/x/y passes.
hipError_t enqueue_step(wdm_plan* p, hipStream_t s, hipStream_t aux, KickMode km,
                        int keep_member = -1) {
    const int prec = p->prec;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) {
        if (e == hipSuccess) e = r;
        return e == hipSuccess;
    };
    for (const auto& c : p->classes) {
        const Launch L{s, p->table, c.first, c.count};
        const bool parts = c.moving_np > 0;
        const bool fork = parts && aux != nullptr;
        if (!chk(timed(p, kKZPot, [&] {
                return launch_z_potential_kick(L, prec, c.nx, c.ny, c.nz, kZKickFft, km,
                                               c.var[kTzPot], c.extended);
            })))
            return e;
        // The particle kernel overlaps the psi passes P2-P4 on the auxiliary
        // stream.  A replayed graph keeps the branch enqueued first on the
        // launching queue and P5 waits on the other one across queues, so the
        // branch expected to take longer goes first: measured at 10^6
        // particles, the particles at 128^3 (particles first 0.118 ms per step,
        // P2 first 0.121 ms) and the psi passes at 256^3 (0.410 and 0.408 ms).
        // The kernels take about 46 ns per 1000 particles and 8 ns per 1000
        // cells for the three passes.
        const bool parts_first = c.moving_np * 6 > int64_t(c.nx) * c.ny * c.nz;
        auto psi_f = [&] {
            return chk(timed(p, kKYPsiF, [&] {
                return launch_y_fft_psi(L, prec, c.nx, c.ny, c.nz, false, c.var[kTyPsi]);
            }));
        };
        if (fork) {
            const Launch LA{aux, p->table, c.first, c.count};
            if (!chk(hipEventRecord(p->ev_fork, s))) return e;
            if (!parts_first && !psi_f()) return e;
            if (!chk(hipStreamWaitEvent(aux, p->ev_fork, 0))) return e;
            if (!chk(timed_on(p, aux, kKParticles, [&] {
                    return launch_particles(LA, prec, c.moving_np, 0, km, p->det,
                                            parts_first ? kPartsAlone : 0);
                })))
                return e;
            if (!chk(hipEventRecord(p->ev_join, aux))) return e;
            if (parts_first && !psi_f()) return e;
        } else {
            if (parts &&
                !chk(timed(p, kKParticles,
                           [&] {
                               return launch_particles(L, prec, c.moving_np, 0, km, p->det,
                                                       kPartsAlone);
                           })))
                return e;
            if (!psi_f()) return e;
        }
        if (!chk(timed(p, kKXKin, [&] {
                return launch_x_kinetic(L, prec, c.nx, c.ny, c.nz, c.var[kTxKin]);
            })))
            return e;
        if (!chk(timed(p, kKYPsiI, [&] {
                return launch_y_fft_psi(L, prec, c.nx, c.ny, c.nz, true, c.var[kTyPsi]);
            })))
            return e;
        if (fork && !chk(hipStreamWaitEvent(s, p->ev_join, 0))) return e;
        if (c.vacuum) {
            if (!chk(enqueue_vacuum_poisson(p, s, c.first, c.count, c.nx, c.ny, c.nz,
                                            kDensInvToPhi)))
                return e;
            continue;
        }
        if (!chk(timed(p, kKZDens, [&] {
                return launch_z_density(L, prec, c.nx, c.ny, c.nz, kDensInvFft, c.var[kTzDens],
                                        keep_member);
            })))
            return e;
        if (!chk(timed(p, kKYSpecF, [&] {
                return launch_y_fft_spec(L, prec, c.nx, c.ny, c.nz, false, c.var[kTySpec]);
            })))
            return e;
        if (!chk(timed(p, kKXGreen, [&] {
                return launch_x_green(L, prec, c.nx, c.ny, c.nz, c.var[kTxGreen]);
            })))
            return e;
        if (!chk(timed(p, kKYSpecI, [&] {
                return launch_y_fft_spec(L, prec, c.nx, c.ny, c.nz, true, c.var[kTySpec]);
            })))
            return e;
    }
    return e;
}

hipError_t enqueue_sort(wdm_plan* p, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (const auto& c : p->classes) {
        if (c.moving_np <= 1) continue;   // static particles keep their order
        e = timed(p, kKSort, [&] {
            return launch_particle_sort(Launch{s, p->table, c.first, c.count}, c.max_np, c.nx,
                                        c.ny, c.nz);
        });
        if (e != hipSuccess) return e;
    }
    return e;
}

hipError_t enqueue_close(wdm_plan* p, hipStream_t s, int64_t n) {
    hipError_t e = hipSuccess;
    for (const auto& c : p->classes) {
        const Launch L{s, p->table, c.first, c.count};
        e = timed(p, kKClose, [&] {
            return launch_z_potential_kick(L, p->prec, c.nx, c.ny, c.nz, kZKickOnly, kHalfKick, 0,
                                           c.extended);
        });
        if (e == hipSuccess && c.moving_np > 0)
            e = timed(p, kKCloseParticles, [&] {
                return launch_particles(L, p->prec, c.moving_np, 1, kHalfKick, p->det);
            });
        if (e == hipSuccess) e = launch_advance_time(L, n);
        if (e == hipSuccess) e = launch_stability(L, watch_slots(c.nx, c.ny), kCKin);
        if (e != hipSuccess) return e;
    }
    return e;
}

bool resort_due(const wdm_plan* p) {
    return p->sort_interval > 0 && p->steps_done > 0 && p->steps_done % p->sort_interval == 0;
}

// Internal streams (default priority) and the fork/join events.
hipError_t ensure_streams(wdm_plan* p) {
    if (p->s_main) return hipSuccess;
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&p->s_main, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipStreamCreateWithFlags(&p->s_aux, hipStreamNonBlocking)) != hipSuccess) return e;
    for (hipEvent_t* ev : {&p->ev_in, &p->ev_out, &p->ev_fork, &p->ev_join})
        if ((e = hipEventCreateWithFlags(ev, hipEventDisableTiming)) != hipSuccess) return e;
    return hipSuccess;
}

// Capture one step (opening or merged) into an executable graph.
hipError_t capture_step(wdm_plan* p, int which) {
    if (p->g_step[which]) return hipSuccess;
    hipError_t e0 = ensure_streams(p);
    if (e0 != hipSuccess) return e0;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(p->s_main, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    for (int i = 0; i < (which == 2 ? kStepChunk : 1) && le == hipSuccess; ++i)
        le = enqueue_step(p, p->s_main, p->s_aux, which ? kFullKick : kHalfKick);
    e = hipStreamEndCapture(p->s_main, &g);
    if (le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(&p->g_step[which], g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

hipError_t enqueue_apply(wdm_net* net, wdm_plan* p, int32_t member, hipStream_t s,
                         bool rho_b_ready);
wdm_status check_net_for(wdm_net* net, wdm_plan* p, int32_t member);

// Capture `every` steps, the closing half kick and the corrector as one graph.
hipError_t capture_block(wdm_plan* p) {
    if (p->g_block) return hipSuccess;
    hipError_t e0 = ensure_streams(p);
    if (e0 != hipSuccess) return e0;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(p->s_main, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    // the last step's P5 keeps the corrected member's baryon deposit (the
    // closing kick moves no particle), so the correction's Poisson rebuild
    // reads it instead of depositing again (periodic members; the vacuum
    // solve clears it)
    const bool keep = p->cfg[p->net_member].boundary != WDM_BOUNDARY_VACUUM;
    const int keep_dev = keep ? p->dev_index[p->net_member] : -1;
    for (int32_t i = 0; i < p->every && le == hipSuccess; ++i)
        le = enqueue_step(p, p->s_main, p->s_aux, i == 0 ? kHalfKick : kFullKick,
                          i + 1 == p->every ? keep_dev : -1);
    if (le == hipSuccess) le = enqueue_close(p, p->s_main, p->every);
    if (le == hipSuccess) le = enqueue_apply(p->net, p, p->net_member, p->s_main, keep);
    e = hipStreamEndCapture(p->s_main, &g);
    if (le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(&p->g_block, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

void drop_graphs(wdm_plan* p) {
    for (hipGraphExec_t& g : p->g_step)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    if (p->g_block) {
        (void)hipGraphExecDestroy(p->g_block);
        p->g_block = nullptr;
    }
}

// What follows a run of steps.
enum After : int { kNoApply = 0, kApplyAfter = 1, kBlockGraph = 2 };

// n steps: opening half kick, n - 1 merged steps, closing half kick, then the
// corrector when `after` asks for it (kBlockGraph: the n = every steps and the
// corrector replayed as the one block graph).
wdm_status run_steps(wdm_plan* p, int64_t n, double dt, After after) {
    const bool graphs = p->use_graphs && !p->profiling;
    if (graphs) {
        bool ok = true;
        for (int w = 0; w < 3 && ok; ++w) ok = capture_step(p, w) == hipSuccess;
        if (ok && after == kBlockGraph) ok = capture_block(p) == hipSuccess;
        if (!ok) {
            drop_graphs(p);
            p->use_graphs = false;   // capture unavailable: launch directly
            (void)hipGetLastError();
            return run_steps(p, n, dt, after == kBlockGraph ? kApplyAfter : after);
        }
    }
    if (after == kBlockGraph && !graphs) after = kApplyAfter;
    // deterministic mode: each call starts from the synchronised state alone,
    // its potential rebuilt as wdm_set_state builds it, so a state saved
    // between calls and set again continues bit for bit
    if (p->det)
        for (int32_t u = 0; u < int32_t(p->cfg.size()); ++u)
            HIPCHK(rebuild_potential(p, u, p->stream));
    // direct launches run on the caller's stream and fork the particle
    // kernel onto the auxiliary stream, as the captured graph does
    HIPCHK(ensure_streams(p));
    hipStream_t s = graphs ? p->s_main : p->stream;
    if (graphs) {
        HIPCHK(hipEventRecord(p->ev_in, p->stream));
        HIPCHK(hipStreamWaitEvent(s, p->ev_in, 0));
    }
    for (const auto& c : p->classes) {
        const Launch L{s, p->table, c.first, c.count};
        HIPCHK(dt != 0.0 ? launch_set_dt(L, dt, 0) : launch_set_dt(L, 0.0, 1));
        HIPCHK(launch_kinetic_tables(L, p->prec, int64_t(c.nx) + int64_t(c.ny) * c.nz));
        if (c.absorb) HIPCHK(launch_absorb_tables(L));
    }
    if (after == kBlockGraph) {
        // a re-sort due inside the block is done before it
        bool due = false;
        for (int64_t i = 0; i < n; ++i) {
            const int64_t k = p->steps_done + i;
            due = due || (p->sort_interval > 0 && k > 0 && k % p->sort_interval == 0);
        }
        if (due) HIPCHK(enqueue_sort(p, s));
        HIPCHK(hipGraphLaunch(p->g_block, s));
        p->steps_done += n;
    } else {
        for (int64_t i = 0; i < n;) {
            if (resort_due(p)) HIPCHK(enqueue_sort(p, s));
            // merged steps up to the end of the run or the next re-sort
            int64_t room = n - i;
            if (p->sort_interval > 0)
                room = std::min<int64_t>(room, p->sort_interval - p->steps_done % p->sort_interval);
            const int64_t k = (graphs && i > 0 && room >= kStepChunk) ? kStepChunk : 1;
            if (graphs)
                HIPCHK(hipGraphLaunch(p->g_step[i == 0 ? 0 : (k > 1 ? 2 : 1)], s));
            else
                HIPCHK(enqueue_step(p, s, p->s_aux, i == 0 ? kHalfKick : kFullKick));
            p->steps_done += k;
            i += k;
        }
        HIPCHK(enqueue_close(p, s, n));
        if (after == kApplyAfter) HIPCHK(enqueue_apply(p->net, p, p->net_member, s, false));
    }
    if (graphs) {
        HIPCHK(hipEventRecord(p->ev_out, s));
        HIPCHK(hipStreamWaitEvent(p->stream, p->ev_out, 0));
    }
    return WDM_OK;
}

}  // namespace

extern "C" {

wdm_status wdm_step(wdm_plan* p, int64_t n, double dt) {
    if (!p) return fail(WDM_EINVAL, "null plan");
    if (n < 0) return fail(WDM_EINVAL, "n must be >= 0");
    if (!std::isfinite(dt)) return fail(WDM_EINVAL, "dt must be finite");
    for (size_t i = 0; i < p->has_state.size(); ++i)
        if (!p->has_state[i]) return fail(WDM_ESTATE, "wdm_set_state not called for every member");
    if (n == 0) return WDM_OK;
    if (!p->net) return run_steps(p, n, dt, kNoApply);
    // with a corrector: runs of steps that end where a correction falls due
    for (int64_t left = n; left > 0;) {
        const int64_t k = std::min<int64_t>(left, p->every - p->corr_phase);
        const bool due = p->corr_phase + k == p->every;
        const After a = !due ? kNoApply : (p->corr_phase == 0 ? kBlockGraph : kApplyAfter);
        if (wdm_status st = run_steps(p, k, dt, a)) return st;
        p->corr_phase = due ? 0 : p->corr_phase + k;
        left -= k;
    }
    return WDM_OK;
}

wdm_status wdm_plan_attach_corrector(wdm_plan* p, wdm_net* net, int32_t member, int32_t every) {
    if (!p) return fail(WDM_EINVAL, "null plan");
    if (!net || every == 0) {   // detach
        if (p->g_block) {
            (void)hipStreamSynchronize(p->stream);
            (void)hipGraphExecDestroy(p->g_block);
            p->g_block = nullptr;
        }
        p->net = nullptr;
        p->every = 0;
        p->corr_phase = 0;
        return WDM_OK;
    }
    if (wdm_status st = check_member(p, member)) return st;
    if (every < 1 || every > 4096) return fail(WDM_EINVAL, "every must be in [1, 4096]");
    if (wdm_status st = check_net_for(net, p, member)) return st;
    if (p->g_block) {
        (void)hipStreamSynchronize(p->stream);
        (void)hipGraphExecDestroy(p->g_block);
        p->g_block = nullptr;
    }
    p->net = net;
    p->net_member = member;
    p->every = every;
    p->corr_phase = 0;
    return WDM_OK;
}

wdm_status wdm_use_graphs(wdm_plan* p, int32_t enable) {
    if (!p) return fail(WDM_EINVAL, "null plan");
    p->use_graphs = enable != 0;
    return WDM_OK;
}

// ---- autotuning of the step passes' FFT plans ------------------------------

namespace {

// Another plan replaces the default only when its median launch time is this
// fraction faster: the plans of one pass are usually within a few per cent,
// and a choice made on noise would change from run to run.
constexpr float kTuneMargin = 0.02f;
// Plans a pass can take: 0 the default, 1 the second radix plan (twice the
// lanes per pencil), 2 (strided passes: y and x) the default radices with
// twice the pencils per work-group, i.e. 256-byte row segments, 3 the default
// radices exchanging whole complex values through LDS (strided passes up to
// 256; z passes where the default splits the exchange).
constexpr int kTunePlans = 4;

// Axis length that decides each tunable pass's plan.
int tune_axis(const SizeClass& c, int slot) {
    switch (slot) {
        case kTzPot: case kTzDens: return c.nz;
        case kTyPsi: case kTySpec: return c.ny;
        default: return c.nx;
    }
}

bool strided_slot(int slot) { return slot != kTzPot && slot != kTzDens; }

// Whether plan v exists for a pass of the class.
bool plan_available(const SizeClass& c, int slot, int v) {
    const int n = tune_axis(c, slot);
    if (v == 0) return true;
    if (v == 1) return axis_has_variant(n);
    if (v == 2) return strided_slot(slot) && axis_has_wide(n);
    return v == 3 && (strided_slot(slot) ? axis_has_wide(n) : axis_has_zcx(n));
}

// One launch of a tunable pass with plan variant v (both directions of the
// y-passes, so a timing covers the pair the step runs).
hipError_t tune_launch(wdm_plan* p, const Launch& L, const SizeClass& c, int slot, int v) {
    hipError_t e;
    switch (slot) {
        case kTzPot:
            return launch_z_potential_kick(L, p->prec, c.nx, c.ny, c.nz, kZKickFft, kFullKick, v);
        case kTyPsi:
            if ((e = launch_y_fft_psi(L, p->prec, c.nx, c.ny, c.nz, false, v)) != hipSuccess) return e;
            return launch_y_fft_psi(L, p->prec, c.nx, c.ny, c.nz, true, v);
        case kTxKin:
            return launch_x_kinetic(L, p->prec, c.nx, c.ny, c.nz, v);
        case kTzDens:
            return launch_z_density(L, p->prec, c.nx, c.ny, c.nz, kDensInvFft, v);
        case kTySpec:
            if ((e = launch_y_fft_spec(L, p->prec, c.nx, c.ny, c.nz, false, v)) != hipSuccess) return e;
            return launch_y_fft_spec(L, p->prec, c.nx, c.ny, c.nz, true, v);
        default:
            return launch_x_green(L, p->prec, c.nx, c.ny, c.nz, v);
    }
}


}  // namespace

int32_t wdm_tuning_entries(const wdm_plan* p) {
    return p ? int32_t(p->classes.size()) * kTuneSlots : 0;
}

wdm_status wdm_get_tuning(wdm_plan* p, int32_t* out, int32_t n) {
    if (!p || !out) return fail(WDM_EINVAL, "null argument");
    if (n != wdm_tuning_entries(p)) return fail(WDM_EINVAL, "n must equal wdm_tuning_entries");
    for (size_t k = 0; k < p->classes.size(); ++k)
        for (int j = 0; j < kTuneSlots; ++j) out[k * kTuneSlots + j] = p->classes[k].var[j];
    return WDM_OK;
}

wdm_status wdm_set_tuning(wdm_plan* p, const int32_t* in, int32_t n) {
    if (!p || !in) return fail(WDM_EINVAL, "null argument");
    if (n != wdm_tuning_entries(p)) return fail(WDM_EINVAL, "n must equal wdm_tuning_entries");
    for (size_t k = 0; k < p->classes.size(); ++k)
        for (int j = 0; j < kTuneSlots; ++j) {
            const int v = in[k * kTuneSlots + j];
            if (v < 0 || v >= kTunePlans)
                return fail(WDM_EINVAL, "plan variants are 0, 1, 2 or 3");
            if (!plan_available(p->classes[k], j, v))
                return fail(WDM_EINVAL, v == 1   ? "no second plan for this axis length"
                                        : v == 2 ? "no wide-row plan for this pass and length"
                                                 : "no complex-exchange plan for this pass and length");
        }
    for (size_t k = 0; k < p->classes.size(); ++k)
        for (int j = 0; j < kTuneSlots; ++j) p->classes[k].var[j] = in[k * kTuneSlots + j];
    drop_graphs(p);
    return WDM_OK;
}

wdm_status wdm_autotune(wdm_plan* p, int32_t reps) {
    if (!p) return fail(WDM_EINVAL, "null plan");
    if (reps < 1 || reps > 1000) return fail(WDM_EINVAL, "reps must be in [1, 1000]");
    if (p->profiling) return fail(WDM_ESTATE, "switch profiling off before tuning");
    // one event pair per timed launch: reps launches of each plan
    std::vector<hipEvent_t> ev(2 * size_t(kTunePlans) * size_t(reps), nullptr);
    auto evp = [&](int r, int v, int w) { return ev[(size_t(r) * kTunePlans + v) * 2 + w]; };
    hipError_t e = hipSuccess;
    for (auto& x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    auto release = [&] {
        for (auto x : ev)
            if (x) (void)hipEventDestroy(x);
    };
    if (e != hipSuccess) {
        release();
        return fail(WDM_EDEVICE, "hipEventCreate failed");
    }
    // the timings run on zeroed fields (FFT timing does not depend on the
    // values); the members' states are overwritten
    for (size_t k = 0; k < p->classes.size() && e == hipSuccess; ++k) {
        SizeClass& c = p->classes[k];
        const Launch L{p->stream, p->table, c.first, c.count};
        const size_t cs = p->prec ? 16 : 8, rs = p->prec ? 8 : 4;
        const int64_t cells = int64_t(c.nx) * c.ny * c.nz;
        for (int d = c.first; d < c.first + c.count && e == hipSuccess; ++d) {
            const MemberDev& m = p->host[d];
            if (e == hipSuccess) e = launch_zero(p->stream, m.psi, size_t(cells) * cs);
            if (e == hipSuccess) e = launch_zero(p->stream, m.phi, size_t(cells) * rs);
            if (e == hipSuccess) e = launch_zero(p->stream, m.rho_b, size_t(cells) * rs);
            if (e == hipSuccess)
                e = launch_zero(p->stream, m.spec, size_t(c.nx) * c.ny * (c.nz / 2) * cs);
            if (e == hipSuccess) e = launch_zero(p->stream, m.spec_nyq, size_t(c.nx) * c.ny * cs);
            if (e == hipSuccess) e = launch_zero(p->stream, m.dt, 4 * sizeof(double));
        }
        for (int j = 0; j < kTuneSlots && e == hipSuccess; ++j) {
            c.var[j] = 0;
            int plans[kTunePlans], np = 0;
            for (int v = 0; v < kTunePlans; ++v)
                if (plan_available(c, j, v)) plans[np++] = v;
            if (np < 2) continue;
            // a warm-up launch of each plan, then reps rounds timing each plan
            // once per round, in rotating order, every launch on its own
            for (int i = 0; i < np && e == hipSuccess; ++i) e = tune_launch(p, L, c, j, plans[i]);
            for (int r = 0; r < reps && e == hipSuccess; ++r)
                for (int q = 0; q < np && e == hipSuccess; ++q) {
                    const int i = (r + q) % np;
                    if ((e = hipEventRecord(evp(r, i, 0), p->stream)) != hipSuccess) break;
                    if ((e = tune_launch(p, L, c, j, plans[i])) != hipSuccess) break;
                    e = hipEventRecord(evp(r, i, 1), p->stream);
                }
            if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
            std::vector<float> t[kTunePlans];
            for (int r = 0; r < reps && e == hipSuccess; ++r)
                for (int i = 0; i < np && e == hipSuccess; ++i) {
                    float ms = 0.0f;
                    e = hipEventElapsedTime(&ms, evp(r, i, 0), evp(r, i, 1));
                    t[i].push_back(ms);
                }
            if (e != hipSuccess) break;
            // medians; another plan must win by kTuneMargin to replace the
            // default, and the fastest such plan is taken
            float med[kTunePlans];
            for (int i = 0; i < np; ++i) {
                std::sort(t[i].begin(), t[i].end());
                const size_t h = t[i].size() / 2;
                med[i] = t[i].size() % 2 ? t[i][h] : 0.5f * (t[i][h - 1] + t[i][h]);
            }
            int best = 0;
            for (int i = 1; i < np; ++i)
                if (med[i] < (1.0f - kTuneMargin) * med[0] && med[i] < med[best]) best = i;
            c.var[j] = plans[best];
        }
    }
    release();
    drop_graphs(p);
    std::fill(p->has_state.begin(), p->has_state.end(), false);
    if (e != hipSuccess) return fail(WDM_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
    return WDM_OK;
}

}  // extern "C"

extern "C" {

wdm_status wdm_get_psi(wdm_plan* p, int32_t member, void* out) {
    if (wdm_status s = check_member(p, member)) return s;
    if (!out) return fail(WDM_EINVAL, "psi_out is null");
    const MemberDev& m = p->host[p->dev_index[member]];
    HIPCHK(hipMemcpyAsync(out, m.psi, size_t(cells_of(p->cfg[member])) * (p->prec ? 16 : 8),
                          hipMemcpyDeviceToDevice, p->stream));
    return WDM_OK;
}

wdm_status wdm_potential(wdm_plan* p, int32_t member, void* out) {
    if (wdm_status s = check_member(p, member)) return s;
    if (!out) return fail(WDM_EINVAL, "phi_out is null");
    if (!p->has_state[member]) return fail(WDM_ESTATE, "no state set");
    const MemberDev& m = p->host[p->dev_index[member]];
    HIPCHK(hipMemcpyAsync(out, m.phi, size_t(cells_of(p->cfg[member])) * (p->prec ? 8 : 4),
                          hipMemcpyDeviceToDevice, p->stream));
    return WDM_OK;
}

wdm_status wdm_density(wdm_plan* p, int32_t member, void* out, int32_t include_baryons) {
    if (wdm_status s = check_member(p, member)) return s;
    if (!out) return fail(WDM_EINVAL, "rho_out is null");
    if (!p->has_state[member]) return fail(WDM_ESTATE, "no state set");
    const wdm_config& c = p->cfg[member];
    const Launch L = one(p, member);
    const MemberDev& m = p->host[p->dev_index[member]];
    const int64_t n = cells_of(c);
    const bool inc = include_baryons && c.n_particles > 0;
    if (inc) {
        HIPCHK(launch_zero(p->stream, m.scratch, size_t(n) * (p->prec ? 8 : 4)));
        HIPCHK(launch_particles(L, p->prec, c.n_particles, 3, kHalfKick, p->det));
    }
    HIPCHK(launch_density_out(L, p->prec, n, out, inc ? 1 : 0));
    return WDM_OK;
}

wdm_status wdm_energy(wdm_plan* p, int32_t member, wdm_energy_t* out) {
    if (wdm_status s = check_member(p, member)) return s;
    if (!out) return fail(WDM_EINVAL, "out is null");
    if (!p->has_state[member]) return fail(WDM_ESTATE, "no state set");
    const wdm_config& c = p->cfg[member];
    const Launch L = one(p, member);
    const MemberDev& m = p->host[p->dev_index[member]];
    const int64_t n = cells_of(c);
    const int prec = p->prec;
    if (wdm_status st = check_stability(p, member)) return st;
    // mass, max |Phi|, max |psi|^2 and sum |psi|^4
    HIPCHK(launch_reduce_grid(L, prec, n, 0));
    HIPCHK(launch_reduce_finish(L, 0, kRedBlocks, false));
    HIPCHK(launch_reduce_finish(L, 7, kRedBlocks, true));
    HIPCHK(launch_reduce_finish(L, 8, kRedBlocks, true));
    HIPCHK(launch_reduce_finish(L, 9, kRedBlocks, false));
    // potential energy with the deposited baryons
    HIPCHK(launch_zero(p->stream, m.scratch, size_t(n) * (prec ? 8 : 4)));
    if (c.n_particles > 0) HIPCHK(launch_particles(L, prec, c.n_particles, 3, kHalfKick, p->det));
    HIPCHK(launch_reduce_grid(L, prec, n, 1));
    HIPCHK(launch_reduce_finish(L, 2, kRedBlocks, false));
    // the stored Phi carries the external potential; its energy enters once
    if (m.ext) {
        HIPCHK(launch_reduce_grid(L, prec, n, 2));
        HIPCHK(launch_reduce_finish(L, 10, kRedBlocks, false));
    }
    // spectral kinetic energy: F_z, F_y into scratch, F_x fused with the sum
    HIPCHK(hipMemcpyAsync(m.scratch, m.psi, size_t(n) * (prec ? 16 : 8), hipMemcpyDeviceToDevice,
                          p->stream));
    HIPCHK(launch_axis_fft(L, prec, c.nx, c.ny, c.nz, 2, false, 1));
    HIPCHK(launch_axis_fft(L, prec, c.nx, c.ny, c.nz, 1, false, 1));
    HIPCHK(launch_x_kinetic_energy(L, prec, c.nx, c.ny, c.nz));
    HIPCHK(launch_reduce_finish(L, 1, int(axis_tiles(c.nx, int64_t(c.ny) * c.nz, prec)), false));
    if (c.n_particles > 0) {
        HIPCHK(launch_reduce_particles(L, c.n_particles));
        for (int f = 3; f < 7; ++f) HIPCHK(launch_reduce_finish(L, f, kRedBlocks, false));
    }
    double res[kRedFields], dts[4], stab[2];
    HIPCHK(hipMemcpyAsync(res, m.results, sizeof(res), hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipMemcpyAsync(dts, m.dt, sizeof(dts), hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipMemcpyAsync(stab, m.stab, sizeof(stab), hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    const double dv = (c.lx / c.nx) * (c.ly / c.ny) * (c.lz / c.nz);
    const double eta = c.hbar_over_m;
    wdm_energy_t r;
    std::memset(&r, 0, sizeof(r));
    r.mass = res[0] * dv;
    r.e_kin = 0.5 * eta * eta * res[1] * dv / double(n);
    const double s_ext = m.ext ? res[10] : 0.0;
    r.e_pot = 0.5 * (res[2] - s_ext) * dv;
    r.e_ext = s_ext * dv;
    if (c.n_particles > 0) {
        r.e_kin_particles = 0.5 * c.particle_mass * res[3];
        for (int a = 0; a < 3; ++a) r.momentum[a] = c.particle_mass * res[4 + a];
    }
    r.e_self = 0.5 * c.kappa * res[9] * dv;
    r.e_total = r.e_kin + r.e_pot + r.e_kin_particles + r.e_self + r.e_ext;
    r.max_abs_phi = res[7];
    r.max_rho = res[8];
    r.t = dts[3];
    r.dt = dts[0] != 0.0 ? dts[0] : dts[1];
    r.dt_auto = dts[1];
    r.cfl_ratio = stab[0];
    const bool finite = std::isfinite(r.mass) && std::isfinite(r.e_total) &&
                        std::isfinite(r.max_abs_phi);
    if (!finite) return fail(WDM_EUNSTABLE, "non-finite state");
    *out = r;
    return WDM_OK;
}

wdm_status wdm_set_external_potential(wdm_plan* p, int32_t member, const void* phi_ext) {
    if (wdm_status s = check_member(p, member)) return s;
    const wdm_config& c = p->cfg[member];
    if (!c.external_potential)
        return fail(WDM_EINVAL, "member was created without external_potential");
    const MemberDev& m = p->host[p->dev_index[member]];
    const int64_t n = cells_of(c);
    const size_t bytes = size_t(n) * (p->prec ? 8 : 4);
    if (phi_ext)
        HIPCHK(hipMemcpyAsync(m.ext, phi_ext, bytes, hipMemcpyDeviceToDevice, p->stream));
    else
        HIPCHK(launch_zero(p->stream, m.ext, bytes));
    HIPCHK(launch_tidal_correct(one(p, member), p->prec, n));
    return WDM_OK;
}

wdm_status wdm_diagnostics(wdm_plan* p, int32_t member, const int32_t* centre,
                           wdm_diagnostics_t* out) {
    if (wdm_status s = check_member(p, member)) return s;
    if (!out) return fail(WDM_EINVAL, "out is null");
    if (!p->has_state[member]) return fail(WDM_ESTATE, "no state set");
    const wdm_config& c = p->cfg[member];
    int cen[3] = {c.nx / 2, c.ny / 2, c.nz / 2};
    if (centre) {
        const int len[3] = {c.nx, c.ny, c.nz};
        for (int a = 0; a < 3; ++a) {
            if (centre[a] < 0 || centre[a] >= len[a])
                return fail(WDM_EINVAL, "centre node out of range");
            cen[a] = centre[a];
        }
    }
    const Launch L = one(p, member);
    const MemberDev& m = p->host[p->dev_index[member]];
    const int64_t n = cells_of(c);
    if (wdm_status st = check_stability(p, member)) return st;
    HIPCHK(launch_diag_energies(L, p->prec, kRedBlocks));
    for (int f = 0; f < 7; ++f) HIPCHK(launch_reduce_finish(L, f, kRedBlocks, false));
    const double dx = c.lx / c.nx;
    const bool cubic = dx == c.ly / c.ny && dx == c.lz / c.nz;
    double radii[9];
    // the histogram and the radii live in the plan's scratch (>= n doubles)
    const int64_t nbins = int64_t(c.nx / 2) * (c.nx / 2) + int64_t(c.ny / 2) * (c.ny / 2) +
                          int64_t(c.nz / 2) * (c.nz / 2) + 1;
    double* hist = static_cast<double*>(m.scratch);
    if (cubic) {
        if (nbins + 9 > n) return fail(WDM_EINVAL, "grid too small for the radial histogram");
        HIPCHK(launch_mass_radii(L, p->prec, n, cen, dx, hist, nbins, hist + nbins));
    }
    double res[kRedFields];
    HIPCHK(hipMemcpyAsync(res, m.results, sizeof(res), hipMemcpyDeviceToHost, p->stream));
    if (cubic)
        HIPCHK(hipMemcpyAsync(radii, hist + nbins, sizeof(radii), hipMemcpyDeviceToHost,
                              p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    const double dv = dx * (c.ly / c.ny) * (c.lz / c.nz);
    out->K = res[0] * dv;
    out->Q = res[1] * dv;
    out->V = res[2] * dv;
    out->virial = 2.0 * out->K + 2.0 * out->Q + out->V;
    for (int a = 0; a < 3; ++a) out->momentum[a] = res[3 + a] * dv;
    out->mass = res[6] * dv;
    for (int f = 0; f < 9; ++f) out->radii[f] = cubic ? radii[f] : std::nan("");
    return WDM_OK;
}

wdm_status wdm_particles(wdm_plan* p, int32_t member, float* pos_out, float* vel_out) {
    if (wdm_status s = check_member(p, member)) return s;
    if (!p->has_state[member]) return fail(WDM_ESTATE, "no state set");
    if (p->cfg[member].n_particles == 0) return WDM_OK;
    HIPCHK(launch_particle_unsort(p->stream, p->host[p->dev_index[member]], pos_out, vel_out));
    return WDM_OK;
}

wdm_status wdm_fft3d(wdm_plan* p, int32_t member, int32_t inverse) {
    if (wdm_status s = check_member(p, member)) return s;
    if (!p->has_state[member]) return fail(WDM_ESTATE, "no state set");
    const wdm_config& c = p->cfg[member];
    const Launch L = one(p, member);
    const bool inv = inverse != 0;
    // forward: z, y, x; inverse: x, y, z
    for (int k = 0; k < 3; ++k)
        HIPCHK(launch_axis_fft(L, p->prec, c.nx, c.ny, c.nz, inv ? k : 2 - k, inv, 0));
    if (inv)
        HIPCHK(launch_scale_complex(p->stream, p->host[p->dev_index[member]].psi, cells_of(c),
                                    1.0 / double(cells_of(c)), p->prec));
    return WDM_OK;
}

wdm_status wdm_set_sort_interval(wdm_plan* p, int32_t interval) {
    if (!p) return fail(WDM_EINVAL, "null plan");
    if (interval < 0) return fail(WDM_EINVAL, "interval must be >= 0");
    p->sort_interval = interval;
    return WDM_OK;
}

wdm_status wdm_profile(wdm_plan* p, int32_t enable) {
    if (!p) return fail(WDM_EINVAL, "null plan");
    p->profiling = enable != 0;
    return WDM_OK;
}

wdm_status wdm_profile_read(wdm_plan* p, wdm_kernel_stat* out, int32_t cap, int32_t* count) {
    if (!p || !count) return fail(WDM_EINVAL, "null argument");
    HIPCHK(hipStreamSynchronize(p->stream));
    if (p->s_aux) HIPCHK(hipStreamSynchronize(p->s_aux));
    std::vector<wdm_kernel_stat> agg(kKinds);
    for (int k = 0; k < kKinds; ++k) {
        std::memset(&agg[k], 0, sizeof(wdm_kernel_stat));
        std::snprintf(agg[k].name, sizeof(agg[k].name), "%s", kKindNames[k]);
    }
    for (const Rec& r : p->recs) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
        agg[r.kind].launches++;
        agg[r.kind].total_ms += ms;
    }
    p->recs.clear();
    p->pool_next = 0;
    int32_t n = 0;
    for (int k = 0; k < kKinds; ++k)
        if (agg[k].launches > 0) {
            if (out && n < cap) out[n] = agg[k];
            ++n;
        }
    *count = n;
    return WDM_OK;
}

wdm_status wdm_copy_bandwidth(void* dst, const void* src, size_t bytes, int32_t reps,
                              void* hip_stream, double* ms_per_copy) {
    if (!dst || !src || !ms_per_copy || reps <= 0 || bytes < 16)
        return fail(WDM_EINVAL, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int64_t n = int64_t(bytes / 16);
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    HIPCHK(launch_stream_copy(s, static_cast<float4*>(dst), static_cast<const float4*>(src), n));
    HIPCHK(hipEventRecord(a, s));
    for (int r = 0; r < reps; ++r)
        HIPCHK(launch_stream_copy(s, static_cast<float4*>(dst), static_cast<const float4*>(src), n));
    HIPCHK(hipEventRecord(b, s));
    HIPCHK(hipEventSynchronize(b));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms_per_copy = double(ms) / reps;
    return WDM_OK;
}

}  // extern "C"

// ===========================================================================
// learned corrector network
// ===========================================================================
namespace {

constexpr int kNetLayers = 3;
constexpr int kNetCin[kNetLayers] = {3, 16, 16};
constexpr int kNetCout[kNetLayers] = {16, 16, 2};
constexpr int kNetCpIn[kNetLayers] = {4, 16, 16};    // padded input channels
constexpr int kNetCpOut[kNetLayers] = {16, 16, 4};   // padded output channels
constexpr int kNetWgradBlocks = 256;

int net_layer_params(int l) { return kNetCout[l] * kNetCin[l] * 27 + kNetCout[l]; }
int net_params() {
    int p = 0;
    for (int l = 0; l < kNetLayers; ++l) p += net_layer_params(l);
    return p;
}
int net_kpad(int cp) { return (27 * cp + 15) / 16 * 16; }

struct NetLayout {
    size_t params, grads, am, av, wf[3], wb[3], x0, a1, a2, y, dy, d2, d1, wpart, wsum[3], dpart,
        mom, scal, total;
};

NetLayout net_layout(int n) {
    const int64_t cells = int64_t(n) * n * n;
    const int P = net_params();
    NetLayout L;
    Carver c;
    L.params = c.take(P * 4);
    L.grads = c.take(P * 4);
    L.am = c.take(P * 4);
    L.av = c.take(P * 4);
    for (int l = 0; l < kNetLayers; ++l) {
        L.wf[l] = c.take(16 * net_kpad(kNetCpIn[l]) * 2);
        L.wb[l] = c.take(16 * net_kpad(kNetCpOut[l]) * 2);
    }
    L.x0 = c.take(cells * 4 * 2);
    L.a1 = c.take(cells * 16 * 2);
    L.a2 = c.take(cells * 16 * 2);
    L.y = c.take(cells * 2 * 4);
    L.dy = c.take(cells * 4 * 2);
    L.d2 = c.take(cells * 16 * 2);
    L.d1 = c.take(cells * 16 * 2);
    L.wpart = c.take(size_t(kNetWgradBlocks) * 16 * wgrad_row(1) * 4);
    for (int l = 0; l < kNetLayers; ++l) L.wsum[l] = c.take(16 * wgrad_row(l) * 4);
    L.dpart = c.take(1024 * 8);
    L.mom = c.take(net_moment_doubles() * 8);
    L.scal = c.take(8 * 8);
    L.total = (c.off + kAlign - 1) / kAlign * kAlign;
    return L;
}

}  // namespace

struct wdm_net {
    hipStream_t stream = nullptr;
    int n = 0;
    int64_t cells = 0;
    uint8_t* ws = nullptr;
    NetLayout L;
    int64_t adam_t = 0;
    bool have_forward = false;
    template <typename T>
    T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
    size_t param_off(int l) const {
        size_t o = 0;
        for (int i = 0; i < l; ++i) o += size_t(net_layer_params(i));
        return o;
    }
};

namespace {

hipError_t net_repack(wdm_net* net) {
    hipError_t e = hipSuccess;
    for (int l = 0; l < kNetLayers && e == hipSuccess; ++l)
        e = net_pack_weights(net->stream, net->at<float>(net->L.params) + net->param_off(l),
                             net->at<uint16_t>(net->L.wf[l]), net->at<uint16_t>(net->L.wb[l]),
                             kNetCin[l], kNetCout[l], kNetCpIn[l], kNetCpOut[l]);
    return e;
}

// The three layers from the packed input x0 (bf16 [cells][4]) on stream s.
hipError_t net_run_layers(wdm_net* net, hipStream_t s) {
    hipError_t e = hipSuccess;
    const uint16_t* in[3] = {net->at<uint16_t>(net->L.x0), net->at<uint16_t>(net->L.a1),
                             net->at<uint16_t>(net->L.a2)};
    void* out[3] = {net->at<uint16_t>(net->L.a1), net->at<uint16_t>(net->L.a2),
                    net->at<float>(net->L.y)};
    for (int l = 0; l < kNetLayers; ++l) {
        const float* b = net->at<float>(net->L.params) + net->param_off(l) +
                         size_t(kNetCout[l]) * kNetCin[l] * 27;
        if ((e = conv_forward_layer(s, l, in[l], net->at<uint16_t>(net->L.wf[l]), b, out[l],
                                    net->n)) != hipSuccess)
            return e;
    }
    return e;
}

// Forward pass of caller inputs x (f32 [cells][3], scaled by the network's
// input scales while packed); y (optional) receives the output.
hipError_t net_run_forward(wdm_net* net, const float* x, float* y) {
    hipStream_t s = net->stream;
    hipError_t e;
    if ((e = net_pack_input(s, x, net->at<uint16_t>(net->L.x0), net->cells, 3, 4,
                            net->at<double>(net->L.scal) + 3)) != hipSuccess)
        return e;
    if ((e = net_run_layers(net, s)) != hipSuccess) return e;
    if (y && y != net->at<float>(net->L.y))
        e = hipMemcpyAsync(y, net->at<float>(net->L.y), size_t(net->cells) * 2 * 4,
                           hipMemcpyDeviceToDevice, s);
    return e;
}

// dy (bf16 [cells][4]) must be in place; accumulates nothing (grads overwritten)
hipError_t net_run_backward(wdm_net* net) {
    hipStream_t s = net->stream;
    hipError_t e;
    const int n = net->n;
    uint16_t* dz[3] = {net->at<uint16_t>(net->L.d1), net->at<uint16_t>(net->L.d2),
                       net->at<uint16_t>(net->L.dy)};
    const uint16_t* act[3] = {net->at<uint16_t>(net->L.x0), net->at<uint16_t>(net->L.a1),
                              net->at<uint16_t>(net->L.a2)};
    for (int l = kNetLayers - 1; l >= 0; --l) {
        if ((e = conv_backward_weight(s, l, dz[l], act[l], net->at<float>(net->L.wpart),
                                      kNetWgradBlocks, net->at<float>(net->L.wsum[l]), n)) !=
            hipSuccess)
            return e;
        float* gw = net->at<float>(net->L.grads) + net->param_off(l);
        float* gb = gw + size_t(kNetCout[l]) * kNetCin[l] * 27;
        if ((e = net_unpack_grads(s, net->at<float>(net->L.wsum[l]), gw, gb, kNetCin[l],
                                  kNetCout[l], kNetCpIn[l], wgrad_row(l))) != hipSuccess)
            return e;
        if (l > 0 &&
            (e = conv_backward_data(s, l, dz[l], net->at<uint16_t>(net->L.wb[l]), act[l],
                                    dz[l - 1], n)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

int32_t wdm_net_param_count(void) { return net_params(); }

size_t wdm_net_workspace_bytes(int32_t n) {
    if (n < 4 || n > 512) {
        g_err = "grid edge must be in [4, 512]";
        return 0;
    }
    return net_layout(n).total;
}

wdm_status wdm_net_create(int32_t n, void* workspace, size_t bytes, void* hip_stream,
                          wdm_net** out) {
    if (!out) return fail(WDM_EINVAL, "out is null");
    *out = nullptr;
    if (n < 4 || n > 512) return fail(WDM_EINVAL, "grid edge must be in [4, 512]");
    const NetLayout L = net_layout(n);
    if (!workspace) return fail(WDM_EINVAL, "workspace is null");
    if (bytes < L.total) return fail(WDM_ENOMEM, "network workspace too small");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
        return fail(WDM_EINVAL, "workspace must be 256-byte aligned");
    auto* net = new wdm_net();
    net->stream = static_cast<hipStream_t>(hip_stream);
    net->n = n;
    net->cells = int64_t(n) * n * n;
    net->ws = static_cast<uint8_t*>(workspace);
    net->L = L;
    const int P = net_params();
    hipError_t e = hipSuccess;
    for (size_t off : {L.params, L.grads, L.am, L.av})   // separately aligned sections
        if (e == hipSuccess) e = launch_zero(net->stream, net->ws + off, size_t(P) * 4);
    if (e == hipSuccess) e = net_repack(net);
    if (e == hipSuccess) e = net_set_scales(net->stream, net->at<double>(L.scal), 1.0, 1.0, 1.0);
    if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
    if (e != hipSuccess) {
        delete net;
        return fail(WDM_EDEVICE, std::string("network initialisation: ") + hipGetErrorString(e));
    }
    *out = net;
    return WDM_OK;
}

wdm_status wdm_net_destroy(wdm_net* net) {
    if (!net) return fail(WDM_EINVAL, "null network");
    (void)hipStreamSynchronize(net->stream);
    delete net;
    return WDM_OK;
}

wdm_status wdm_net_set_params(wdm_net* net, const float* params) {
    if (!net || !params) return fail(WDM_EINVAL, "null argument");
    HIPCHK(hipMemcpy(net->ws + net->L.params, params, size_t(net_params()) * 4,
                     hipMemcpyHostToDevice));
    HIPCHK(launch_zero(net->stream, net->ws + net->L.am, size_t(net_params()) * 4));
    HIPCHK(launch_zero(net->stream, net->ws + net->L.av, size_t(net_params()) * 4));
    net->adam_t = 0;
    HIPCHK(net_repack(net));
    return WDM_OK;
}

wdm_status wdm_net_get_params(wdm_net* net, float* params) {
    if (!net || !params) return fail(WDM_EINVAL, "null argument");
    HIPCHK(hipStreamSynchronize(net->stream));
    HIPCHK(hipMemcpy(params, net->ws + net->L.params, size_t(net_params()) * 4,
                     hipMemcpyDeviceToHost));
    return WDM_OK;
}

wdm_status wdm_net_get_grads(wdm_net* net, float* grads) {
    if (!net || !grads) return fail(WDM_EINVAL, "null argument");
    HIPCHK(hipStreamSynchronize(net->stream));
    HIPCHK(hipMemcpy(grads, net->ws + net->L.grads, size_t(net_params()) * 4,
                     hipMemcpyDeviceToHost));
    return WDM_OK;
}

wdm_status wdm_net_forward(wdm_net* net, const float* x, float* y) {
    if (!net || !x) return fail(WDM_EINVAL, "null argument");
    HIPCHK(net_run_forward(net, x, y));
    net->have_forward = true;
    return WDM_OK;
}

wdm_status wdm_net_backward(wdm_net* net, const float* dy) {
    if (!net || !dy) return fail(WDM_EINVAL, "null argument");
    if (!net->have_forward) return fail(WDM_ESTATE, "backward needs a forward pass first");
    HIPCHK(net_pack_input(net->stream, dy, net->at<uint16_t>(net->L.dy), net->cells, 2, 4,
                          nullptr));
    HIPCHK(net_run_backward(net));
    return WDM_OK;
}

wdm_status wdm_net_mse_backward(wdm_net* net, const float* target, double* loss) {
    if (!net || !target) return fail(WDM_EINVAL, "null argument");
    if (!net->have_forward) return fail(WDM_ESTATE, "backward needs a forward pass first");
    double* scal = net->at<double>(net->L.scal);
    HIPCHK(net_mse(net->stream, net->at<float>(net->L.y), target, net->at<uint16_t>(net->L.dy),
                   net->at<double>(net->L.dpart), scal, net->cells, 2, 4, scal + 5));
    HIPCHK(net_run_backward(net));
    if (loss) {
        HIPCHK(hipMemcpyAsync(loss, scal, sizeof(double), hipMemcpyDeviceToHost, net->stream));
        HIPCHK(hipStreamSynchronize(net->stream));
    }
    return WDM_OK;
}

wdm_status wdm_net_adam(wdm_net* net, double lr, double b1, double b2, double eps) {
    if (!net) return fail(WDM_EINVAL, "null network");
    if (!(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
        return fail(WDM_EINVAL, "bad Adam hyper-parameters");
    net->adam_t++;
    const double c1 = 1.0 - std::pow(b1, double(net->adam_t));
    const double c2 = 1.0 - std::pow(b2, double(net->adam_t));
    HIPCHK(net_adam(net->stream, net->at<float>(net->L.params), net->at<float>(net->L.grads),
                    net->at<float>(net->L.am), net->at<float>(net->L.av), net_params(), float(lr),
                    float(b1), float(b2), float(eps), float(c1), float(c2)));
    HIPCHK(net_repack(net));
    return WDM_OK;
}

wdm_status wdm_net_set_scales(wdm_net* net, double s_psi, double s_phi, double s_out) {
    if (!net) return fail(WDM_EINVAL, "null network");
    if (!(std::isfinite(s_psi) && std::isfinite(s_phi) && std::isfinite(s_out)))
        return fail(WDM_EINVAL, "scales must be finite");
    HIPCHK(net_set_scales(net->stream, net->at<double>(net->L.scal), s_psi, s_phi, s_out));
    return WDM_OK;
}

wdm_status wdm_net_get_scales(wdm_net* net, double* out) {
    if (!net || !out) return fail(WDM_EINVAL, "null argument");
    double sc[8];
    HIPCHK(hipMemcpyAsync(sc, net->at<double>(net->L.scal), sizeof(sc), hipMemcpyDeviceToHost,
                          net->stream));
    HIPCHK(hipStreamSynchronize(net->stream));
    for (int i = 0; i < 3; ++i) out[i] = sc[3 + i];
    return WDM_OK;
}

wdm_status wdm_net_fit_scales(wdm_net* net, const float* const* xs, const float* const* ys,
                              int32_t count) {
    if (!net || !xs || !ys || count < 1) return fail(WDM_EINVAL, "need count >= 1 pairs");
    for (int32_t i = 0; i < count; ++i)
        if (!xs[i] || !ys[i]) return fail(WDM_EINVAL, "null pair buffer");
    double* rows = net->at<double>(net->L.mom);
    for (int32_t i = 0; i < count; ++i)
        HIPCHK(net_moments(net->stream, xs[i], ys[i], net->cells, rows, i == 0));
    HIPCHK(net_fit_scales(net->stream, rows, double(count) * double(net->cells),
                          net->at<double>(net->L.scal)));
    return WDM_OK;
}

}  // extern "C"

namespace {

// The corrector on a member's synchronised state, on stream s: network inputs
// from (psi, Phi) with the network's scales, the three layers, psi += s_out y,
// psi rescaled to its FP64 mass before the correction, and the potential
// rebuilt from the corrected state (moving particles redeposited).
hipError_t enqueue_apply(wdm_net* net, wdm_plan* p, int32_t member, hipStream_t s,
                         bool rho_b_ready) {
    const MemberDev& m = p->host[p->dev_index[member]];
    float* psi = static_cast<float*>(m.psi);
    double* scal = net->at<double>(net->L.scal);
    double* part = net->at<double>(net->L.dpart);
    hipError_t e;
    if ((e = net_state_pack(s, psi, static_cast<const float*>(m.phi),
                            net->at<uint16_t>(net->L.x0), net->cells, scal, part)) != hipSuccess)
        return e;
    // the first two layers, then the last one with psi += s_out d in its
    // epilogue; the mass restoration rides on the rebuild's density pass
    // (periodic members)
    const uint16_t* in[2] = {net->at<uint16_t>(net->L.x0), net->at<uint16_t>(net->L.a1)};
    uint16_t* out[2] = {net->at<uint16_t>(net->L.a1), net->at<uint16_t>(net->L.a2)};
    auto bias = [&](int l) {
        return net->at<float>(net->L.params) + net->param_off(l) +
               size_t(kNetCout[l]) * kNetCin[l] * 27;
    };
    for (int l = 0; l < 2; ++l)
        if ((e = conv_forward_layer(s, l, in[l], net->at<uint16_t>(net->L.wf[l]), bias(l), out[l],
                                    net->n)) != hipSuccess)
            return e;
    const bool periodic = p->cfg[member].boundary != WDM_BOUNDARY_VACUUM;
    if ((e = net_last_layer_apply(s, net->at<uint16_t>(net->L.a2),
                                  net->at<uint16_t>(net->L.wf[2]), bias(2), psi, net->n, scal,
                                  part, !periodic)) != hipSuccess)
        return e;
    return rebuild_potential(p, member, s, rho_b_ready, periodic ? scal : nullptr);
}

// Checks shared by wdm_net_apply and wdm_plan_attach_corrector.
wdm_status check_net_for(wdm_net* net, wdm_plan* p, int32_t member) {
    const wdm_config& c = p->cfg[member];
    if (p->prec != WDM_C64) return fail(WDM_EUNSUPPORTED, "corrector needs a complex64 plan");
    if (c.nx != net->n || c.ny != net->n || c.nz != net->n)
        return fail(WDM_EINVAL, "network grid differs from the member's grid");
    if (net->stream != p->stream) return fail(WDM_EINVAL, "network and plan must share a stream");
    return WDM_OK;
}

}  // namespace

extern "C" {

wdm_status wdm_net_apply(wdm_net* net, wdm_plan* p, int32_t member) {
    if (!net) return fail(WDM_EINVAL, "null network");
    if (wdm_status st = check_member(p, member)) return st;
    if (wdm_status st = check_net_for(net, p, member)) return st;
    if (!p->has_state[member]) return fail(WDM_ESTATE, "no state set");
    HIPCHK(enqueue_apply(net, p, member, p->stream, false));
    return WDM_OK;
}

wdm_status wdm_net_pair(wdm_plan* p, int32_t member, const void* target, float* x_out,
                        float* y_out) {
    if (wdm_status st = check_member(p, member)) return st;
    if (!target || !x_out || !y_out) return fail(WDM_EINVAL, "null argument");
    if (p->prec != WDM_C64) return fail(WDM_EUNSUPPORTED, "training pairs need a complex64 plan");
    if (!p->has_state[member]) return fail(WDM_ESTATE, "no state set");
    const MemberDev& m = p->host[p->dev_index[member]];
    HIPCHK(net_pair(p->stream, static_cast<const float*>(m.psi), static_cast<const float*>(m.phi),
                    static_cast<const float*>(target), x_out, y_out, cells_of(p->cfg[member])));
    return WDM_OK;
}

}  // extern "C"

// ===========================================================================
// spectral utilities: restriction and shell power spectrum
// ===========================================================================
extern "C" {

wdm_status wdm_restrict(wdm_plan* fine, int32_t fmember, wdm_plan* coarse, int32_t cmember,
                        void* psi_out) {
    if (wdm_status st = check_member(fine, fmember)) return st;
    if (wdm_status st = check_member(coarse, cmember)) return st;
    if (!psi_out) return fail(WDM_EINVAL, "psi_out is null");
    const wdm_config& f = fine->cfg[fmember];
    const wdm_config& c = coarse->cfg[cmember];
    if (f.nx != f.ny || f.nx != f.nz || c.nx != c.ny || c.nx != c.nz)
        return fail(WDM_EUNSUPPORTED, "restriction needs cubic grids");
    if (c.nx >= f.nx) return fail(WDM_EINVAL, "the coarse grid must be smaller");
    if (fine->prec != coarse->prec) return fail(WDM_EINVAL, "plans must share a precision");
    if (fine->stream != coarse->stream) return fail(WDM_EINVAL, "plans must share a stream");
    if (!fine->has_state[fmember]) return fail(WDM_ESTATE, "no state set on the fine member");
    const int prec = fine->prec;
    const MemberDev& mf = fine->host[fine->dev_index[fmember]];
    const MemberDev& mc = coarse->host[coarse->dev_index[cmember]];
    const Launch LF = one(fine, fmember), LC = one(coarse, cmember);
    const size_t cs = prec ? 16 : 8;
    HIPCHK(hipMemcpyAsync(mf.scratch, mf.psi, size_t(cells_of(f)) * cs, hipMemcpyDeviceToDevice,
                          fine->stream));
    for (int ax = 2; ax >= 0; --ax)
        HIPCHK(launch_axis_fft(LF, prec, f.nx, f.ny, f.nz, ax, false, 1));
    HIPCHK(launch_restrict_modes(fine->stream, mf.scratch, mc.scratch, f.nx, c.nx, prec));
    for (int ax = 0; ax < 3; ++ax)
        HIPCHK(launch_axis_fft(LC, prec, c.nx, c.ny, c.nz, ax, true, 1));
    HIPCHK(hipMemcpyAsync(psi_out, mc.scratch, size_t(cells_of(c)) * cs, hipMemcpyDeviceToDevice,
                          coarse->stream));
    return WDM_OK;
}

wdm_status wdm_distance(wdm_plan* p, int32_t member, const void* other, double* out) {
    if (wdm_status st = check_member(p, member)) return st;
    if (!other || !out) return fail(WDM_EINVAL, "null argument");
    if (!p->has_state[member]) return fail(WDM_ESTATE, "no state set");
    const MemberDev& m = p->host[p->dev_index[member]];
    // 2 x 1024 partials and the two sums at the end of the reduction staging
    double* part = m.partials;
    double* res = m.partials + 2 * 1024;
    HIPCHK(launch_distance(one(p, member), p->prec, other, cells_of(p->cfg[member]), part, res));
    double host[2];
    HIPCHK(hipMemcpyAsync(host, res, sizeof(host), hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    out[0] = host[0];
    out[1] = host[1];
    return WDM_OK;
}

wdm_status wdm_power_spectrum(wdm_plan* p, int32_t member, int32_t nbins, double* pk,
                              int64_t* counts) {
    if (wdm_status st = check_member(p, member)) return st;
    if (!pk || nbins < 1 || nbins > 1024) return fail(WDM_EINVAL, "need 1 <= nbins <= 1024");
    const wdm_config& c = p->cfg[member];
    if (c.nx != c.ny || c.nx != c.nz) return fail(WDM_EUNSUPPORTED, "P(k) needs a cubic grid");
    if (!p->has_state[member]) return fail(WDM_ESTATE, "no state set");
    const Launch L = one(p, member);
    const int64_t n = cells_of(c);
    HIPCHK(launch_reduce_grid(L, p->prec, n, 0));
    HIPCHK(launch_reduce_finish(L, 0, kRedBlocks, false));
    HIPCHK(launch_contrast(L, p->prec, n));
    for (int ax = 2; ax >= 0; --ax)
        HIPCHK(launch_axis_fft(L, p->prec, c.nx, c.ny, c.nz, ax, false, 1));
    double* part = reinterpret_cast<double*>(p->ws + p->layout.pk);
    double* res = part + shells_partial_doubles() - 2 * 1024;
    HIPCHK(launch_shells(L, p->prec, nbins, part, res));
    std::vector<double> host(2 * size_t(nbins));
    HIPCHK(hipMemcpyAsync(host.data(), res, host.size() * sizeof(double), hipMemcpyDeviceToHost,
                          p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    for (int b = 0; b < nbins; ++b) {
        const double cnt = host[nbins + b];
        pk[b] = cnt > 0 ? host[b] / cnt : 0.0;
        if (counts) counts[b] = int64_t(cnt);
    }
    return WDM_OK;
}

}  // extern "C"
