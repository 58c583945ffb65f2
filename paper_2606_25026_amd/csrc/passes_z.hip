// P1 and P5: the passes along the contiguous z axis.
#include "passes_common.hpp"

namespace wdm {

// Absorbing factors of one pencil for the extended kick: b_x b_y of the pencil
// (returned) and the z factors staged in LDS, all loads issued with the
// pass's other loads.  Ones when the member has no absorbing boundary.
template <int NZ, int WG>
__device__ __forceinline__ double load_absorb(double* bz, const MemberDev& m, int64_t q, bool ok) {
    constexpr int R = (NZ + WG - 1) / WG;
    if (m.absorb_alpha == 0.0) return 1.0;
    const double* tz = m.absorb + m.nx + m.ny;
    double r[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = int(threadIdx.x) + k * WG;
        r[k] = (NZ % WG == 0 || i < NZ) ? gldr(tz, i) : 1.0;
    }
    double bxy = 1.0;
    if (ok) {
        const int64_t i = q / m.ny, j = q - i * m.ny;
        bxy = gldr(m.absorb, i) * gldr(m.absorb, m.nx + j);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = int(threadIdx.x) + k * WG;
        if (NZ % WG == 0 || i < NZ) bz[i] = r[k];
    }
    return bxy;
}

// Kick with the local self-interaction and the absorbing boundary (Sec. 2.2,
// 3.1): the potential is V = Phi + kappa |psi|^2, taken from psi before the
// kick (the kick keeps |psi|).  With MASK the absorbing factor
// B = b_x b_y b_z closes the step; in a merged kick (FULL) it falls between
// the closing half kick of one step and the opening one of the next, whose
// self-interaction then sees |B psi|^2:
//   phase = -dt/eta (Phi + kappa |psi|^2 (1 + B^2) / 2),  psi <- B e^{i phase} psi.
// `c` is -tau / eta of the kick as launched; `bxy` and `bz` come from
// load_absorb.
template <class FP, typename T, bool MASK, bool FULL, class LN>
__device__ __forceinline__ void kick_general(cplx<T>* v, const cplx<T>* w, const T* phi,
                                             const MemberDev& m, double bxy, const double* bz,
                                             double c, const LN& ln) {
    const double kappa = m.kappa;
    const bool mask = MASK && m.absorb_alpha != 0.0;
#pragma unroll
    for (int s = 0; s < FP::E; ++s) {
        const double re = double(w[s].re), im = double(w[s].im);
        const double r2 = re * re + im * im;
        const double b = mask ? bxy * bz[slot_elem<FP, FP::first()>(ln.t, s)] : 1.0;
        const double pot = double(phi[s]) + kappa * r2 * (FULL ? 0.5 * (1.0 + b * b) : 1.0);
        cplx<T> r = rotate(w[s], pot * c);
        if (mask) {
            r.re *= T(b);
            r.im *= T(b);
        }
        v[s] = r;
    }
}

// ===========================================================================
// P1: potential from the half spectrum, kick, optional forward z-FFT.
// ===========================================================================
// GEN selects the kick with self-interaction and absorbing boundary (kept out
// of the plain kernel, whose register budget it would otherwise raise).
template <int NZ, typename T, int OP, int KICK, int V, bool GEN>
__global__ __launch_bounds__((wg_size<typename PlanFor<NZ, V>::type, T>())) void k_z_potential_kick(
    const MemberDev* __restrict__ mems, int first) {
    using FP = typename PlanFor<NZ, V>::type;
    using IP = Reversed<FP>;
    using LN = Lanes<FP, T, false>;
    constexpr int PP = LN::PP;
    constexpr int H = NZ / 2;
    // the closing kick and the merged kick end a step: the absorbing boundary
    // follows them; the opening kick has none before it
    constexpr bool MASK = GEN && (OP == kZKickOnly || KICK == kFullKick);
    // real entries for a split exchange, complex ones otherwise
    __shared__ lds_t<FP, T, false> lds[lds_entries<FP, T, false>()];
    __shared__ cplx<T> tw[tw_entries<T>(NZ)];
    __shared__ double bz[MASK ? NZ : 1];
    const MemberDev& m = mems[first + blockIdx.y];
    const LN ln;
    const int64_t npen = int64_t(m.nx) * m.ny;
    const int64_t q = int64_t(blockIdx.x) * PP + ln.p;
    const bool ok = q < npen;
    load_twiddles<NZ, wg_size<FP, T>()>(tw, m.tw_z);
    double bxy = 1.0;
    if constexpr (MASK) bxy = load_absorb<NZ, wg_size<FP, T>()>(bz, m, q, ok);
    // psi is loaded together with the spectrum: one memory wait per pass
    cplx<T>* psi = static_cast<cplx<T>*>(m.psi);
    cplx<T> w[OP == kZPhiOnly ? 1 : FP::E];
    if constexpr (OP != kZPhiOnly) load_slots<FP, FP::first()>(w, psi, q * NZ, 1, ok, ln);
    // half spectrum e in [0, H) (H / T per lane) and the Nyquist element e = H,
    // all loads issued before the LDS writes
    static_assert(H % FP::T == 0, "half pencil must split evenly over the lanes");
    constexpr int HE = H / FP::T;
    const cplx<T>* spec = static_cast<const cplx<T>*>(m.spec) + q * H + ln.t;
    cplx<T> hs[HE + 1];
#pragma unroll
    for (int k = 0; k < HE; ++k) hs[k] = ok ? gld(spec, k * FP::T) : cplx<T>{T(0), T(0)};
    hs[HE] = (ok && ln.t == 0) ? gld(static_cast<const cplx<T>*>(m.spec_nyq), q)
                               : cplx<T>{T(0), T(0)};
    // Hermitian completion F[e] = conj(F[NZ - e]) for e > NZ/2, in the input
    // layout of the inverse plan (with the split exchange: real parts, then
    // imaginary parts, through LDS)
    cplx<T> v[FP::E];
    if constexpr (split_exchange<FP, false>()) {
#pragma unroll
        for (int part = 0; part < 2; ++part) {
#pragma unroll
            for (int k = 0; k < HE; ++k) lds[ln(ln.t + k * FP::T)] = part ? hs[k].im : hs[k].re;
            if (ln.t == 0) lds[ln(H)] = part ? hs[HE].im : hs[HE].re;
            __syncthreads();
#pragma unroll
            for (int s = 0; s < FP::E; ++s) {
                const int e = slot_elem<IP, IP::first()>(ln.t, s);
                const T x = e <= H ? lds[ln(e)] : lds[ln(NZ - e)];
                if (part)
                    v[s].im = e <= H ? x : -x;
                else
                    v[s].re = x;
            }
            __syncthreads();
        }
    } else {
#pragma unroll
        for (int k = 0; k < HE; ++k) lds[ln(ln.t + k * FP::T)] = hs[k];
        if (ln.t == 0) lds[ln(H)] = hs[HE];
        __syncthreads();
#pragma unroll
        for (int s = 0; s < FP::E; ++s) {
            const int e = slot_elem<IP, IP::first()>(ln.t, s);
            v[s] = e <= H ? lds[ln(e)] : conj(lds[ln(NZ - e)]);
        }
        __syncthreads();
    }
    pencil_fft<IP, true, T>(v, lds, tw, ln.t, ln);
    // output layout of IP == input layout of FP
    T phi[FP::E];
    T* gphi = static_cast<T*>(m.phi) + q * NZ;
#pragma unroll
    for (int s = 0; s < FP::E; ++s) phi[s] = v[s].re;
    if constexpr (GEN) {
        // an external potential joins the self-gravity felt by the wave and,
        // through the stored Phi, by the particles; loaded here rather than
        // with the other loads, so only runs that have one pay the wait
        if (m.ext != nullptr && ok) {
            const T* ge = static_cast<const T*>(m.ext) + q * NZ;
#pragma unroll
            for (int s = 0; s < FP::E; ++s) phi[s] += gldr(ge, slot_elem<FP, FP::first()>(ln.t, s));
        }
    }
#pragma unroll
    for (int s = 0; s < FP::E; ++s)
        if (ok) gstr(gphi, slot_elem<FP, FP::first()>(ln.t, s), phi[s]);
    // lanes past the last pencil hold zeros here
    watch_max<FP::E>(m.watch, m.watch_n, phi);
    if constexpr (OP == kZPhiOnly) return;
    const double dt = gldr(m.dt, 0);
    const double tau = (KICK == kFullKick) ? dt : 0.5 * dt;
    const double c = -tau / m.eta;
    if constexpr (GEN) {
        if (m.kappa != 0.0) {
            // |psi|^2 before the kick: the self-interaction's CFL term
            T r2[FP::E];
#pragma unroll
            for (int s = 0; s < FP::E; ++s) r2[s] = ok ? w[s].re * w[s].re + w[s].im * w[s].im : T(0);
            watch_max<FP::E>(m.watch + m.watch_n, m.watch_n, r2);
        }
        kick_general<FP, T, MASK, KICK == kFullKick>(v, w, phi, m, bxy, bz, c, ln);
    } else {
#pragma unroll
        for (int s = 0; s < FP::E; ++s) v[s] = rotate(w[s], double(phi[s]) * c);
    }
    if constexpr (OP == kZKickOnly) {
        store_slots<FP, FP::first()>(v, psi, q * NZ, 1, ok, ln);
        return;
    }
    __syncthreads();
    pencil_fft<FP, false, T>(v, lds, tw, ln.t, ln);
    store_slots<FP, FP::last()>(v, psi, q * NZ, 1, ok, ln);
}


// ===========================================================================
// P5: inverse z-FFT of psi, density, R2C forward z-FFT into the half spectrum.
// ===========================================================================
// `keep`: the device index of a member whose rho_b is left in place (the
// Poisson rebuild after a correction of that member reads it instead of
// depositing the unchanged positions again), -1 for none.  `scal` (direct density
// only, else null): psi is first scaled by sqrt(scal[1] / scal[2]) and written
// back -- the corrector's mass restoration, fused into the rebuild that reads
// psi anyway.
template <int NZ, typename T, int OP, int V>
__global__ __launch_bounds__((wg_size<typename PlanFor<NZ, V>::type, T>())) void k_z_density(
    const MemberDev* __restrict__ mems, int first, int keep, const double* __restrict__ scal) {
    using FP = typename PlanFor<NZ, V>::type;
    using IP = Reversed<FP>;
    using LN = Lanes<FP, T, false>;
    constexpr int PP = LN::PP;
    constexpr int H = NZ / 2;
    constexpr bool INV = OP == kDensInvFft || OP == kDensInvToPhi;
    constexpr bool TO_PHI = OP == kDensInvToPhi || OP == kDensDirectToPhi;
    constexpr bool FROM_PHI = OP == kPhiR2C;
    // real entries for a split exchange, complex ones otherwise
    __shared__ lds_t<FP, T, false> lds[lds_entries<FP, T, false>()];
    __shared__ cplx<T> tw[tw_entries<T>(NZ)];
    const MemberDev& m = mems[first + blockIdx.y];
    const LN ln;
    const int64_t npen = int64_t(m.nx) * m.ny;
    const int64_t q = int64_t(blockIdx.x) * PP + ln.p;
    const bool ok = q < npen;
    load_twiddles<NZ, wg_size<FP, T>()>(tw, m.tw_z);
    cplx<T>* psi = static_cast<cplx<T>*>(m.psi);
    T* ph = static_cast<T*>(m.phi) + q * NZ + ln.t;
    cplx<T> v[FP::E];
    // the baryon density is loaded after psi's inverse transform: held across
    // the transform it cost more registers (85 against 72 at 256, five waves
    // per SIMD against seven) than the second memory wait costs
    T* rb = static_cast<T*>(m.rho_b) + q * NZ + ln.t;
    T rbv[FP::E];
    // a member without particles has no baryon density: rho_b stays zero and
    // is neither read nor cleared
    const bool touched = ok && m.np > 0;
    if constexpr (FROM_PHI) {
#pragma unroll
        for (int s = 0; s < FP::E; ++s)
            v[s] = cplx<T>{ok ? gldr(ph, slot_const<FP, FP::first()>(s)) : T(0), T(0)};
        __syncthreads();
    } else {
        if constexpr (INV) {
            load_slots<IP, IP::first()>(v, psi, q * NZ, 1, ok, ln);
            __syncthreads();
            pencil_fft<IP, true, T>(v, lds, tw, ln.t, ln);
            store_slots<FP, FP::first()>(v, psi, q * NZ, 1, ok, ln);
        } else {
            load_slots<FP, FP::first()>(v, psi, q * NZ, 1, ok, ln);
            if constexpr (OP == kDensDirect) {
                if (scal != nullptr) {
                    const double a = gldr(scal, 2);
                    const T f = a > 0.0 ? T(sqrt(gldr(scal, 1) / a)) : T(1);
#pragma unroll
                    for (int s = 0; s < FP::E; ++s) v[s] = cplx<T>{v[s].re * f, v[s].im * f};
                    store_slots<FP, FP::first()>(v, psi, q * NZ, 1, ok, ln);
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int s = 0; s < FP::E; ++s)
            rbv[s] = touched ? gldr(rb, slot_const<FP, FP::first()>(s)) : T(0);
        // the accumulator is cleared for the next deposit; a static deposit stays
        const bool clear = touched && !m.static_baryons && first + int(blockIdx.y) != keep;
#pragma unroll
        for (int s = 0; s < FP::E; ++s) {
            v[s] = cplx<T>{v[s].re * v[s].re + v[s].im * v[s].im + rbv[s], T(0)};
            if (clear) gstr(rb, slot_const<FP, FP::first()>(s), T(0));
        }
        if constexpr (TO_PHI) {
            if (ok) {
#pragma unroll
                for (int s = 0; s < FP::E; ++s) gstr(ph, slot_const<FP, FP::first()>(s), v[s].re);
            }
            return;
        }
    }
    __syncthreads();
    pencil_fft<FP, false, T>(v, lds, tw, ln.t, ln);
    if (!ok) return;
    cplx<T>* spec = static_cast<cplx<T>*>(m.spec) + q * H;
#pragma unroll
    for (int s = 0; s < FP::E; ++s) {
        const int e = slot_elem<FP, FP::last()>(ln.t, s);
        if (e < H)
            gst(spec, e, v[s]);
        else if (e == H)
            gst(static_cast<cplx<T>*>(m.spec_nyq), q, v[s]);
    }
}


bool axis_has_zcx(int n) { return axis_supported(n) && has_zcx(n); }

template <int NZ>
struct ZPotKick {
    template <typename T, int V, bool GEN>
    static hipError_t go(const Launch& L, int nx, int ny, ZOp op, KickMode k) {
        dim3 grid(unsigned(tiles<NZ, T, V>(int64_t(nx) * ny)), unsigned(L.count));
        const dim3 b = block<NZ, T, V>();
        if constexpr (V == 0) {
            if (op == kZPhiOnly) {
                k_z_potential_kick<NZ, T, kZPhiOnly, kHalfKick, 0, GEN>
                    <<<grid, b, 0, L.stream>>>(L.members, L.first);
                return hipGetLastError();
            }
            if (op == kZKickOnly) {
                if (k == kHalfKick)
                    k_z_potential_kick<NZ, T, kZKickOnly, kHalfKick, 0, GEN>
                        <<<grid, b, 0, L.stream>>>(L.members, L.first);
                else
                    k_z_potential_kick<NZ, T, kZKickOnly, kFullKick, 0, GEN>
                        <<<grid, b, 0, L.stream>>>(L.members, L.first);
                return hipGetLastError();
            }
        }
        if (k == kHalfKick)
            k_z_potential_kick<NZ, T, kZKickFft, kHalfKick, V, GEN>
                <<<grid, b, 0, L.stream>>>(L.members, L.first);
        else
            k_z_potential_kick<NZ, T, kZKickFft, kFullKick, V, GEN>
                <<<grid, b, 0, L.stream>>>(L.members, L.first);
        return hipGetLastError();
    }
    template <typename T>
    static hipError_t pick(const Launch& L, int nx, int ny, ZOp op, KickMode k, int var,
                           bool gen) {
        // the extended kick runs on the default plan only
        if (gen) return go<T, 0, true>(L, nx, ny, op, k);
        // only the merged kick + z-FFT variant has other plans
        if constexpr (has_variant(NZ))
            if (var == 1 && op == kZKickFft) return go<T, 1, false>(L, nx, ny, op, k);
        if constexpr (has_zcx(NZ))
            if (var == 3 && op == kZKickFft) return go<T, 3, false>(L, nx, ny, op, k);
        return go<T, 0, false>(L, nx, ny, op, k);
    }
    static hipError_t run(const Launch& L, int prec, int nx, int ny, ZOp op, KickMode k, int var,
                          bool gen) {
        return prec ? pick<double>(L, nx, ny, op, k, var, gen)
                    : pick<float>(L, nx, ny, op, k, var, gen);
    }
};

template <int NZ>
struct ZDens {
    template <typename T, int V>
    static hipError_t go(const Launch& L, int nx, int ny, DensOp op, int keep,
                         const double* scal) {
        dim3 grid(unsigned(tiles<NZ, T, V>(int64_t(nx) * ny)), unsigned(L.count));
        const dim3 b = block<NZ, T, V>();
        if constexpr (V == 0) {
            switch (op) {
                case kDensDirect:
                    k_z_density<NZ, T, kDensDirect, 0>
                        <<<grid, b, 0, L.stream>>>(L.members, L.first, keep, scal);
                    return hipGetLastError();
                case kDensInvToPhi:
                    k_z_density<NZ, T, kDensInvToPhi, 0>
                        <<<grid, b, 0, L.stream>>>(L.members, L.first, keep, scal);
                    return hipGetLastError();
                case kDensDirectToPhi:
                    k_z_density<NZ, T, kDensDirectToPhi, 0>
                        <<<grid, b, 0, L.stream>>>(L.members, L.first, keep, scal);
                    return hipGetLastError();
                case kPhiR2C:
                    k_z_density<NZ, T, kPhiR2C, 0>
                        <<<grid, b, 0, L.stream>>>(L.members, L.first, keep, scal);
                    return hipGetLastError();
                default:
                    break;
            }
        }
        k_z_density<NZ, T, kDensInvFft, V>
            <<<grid, b, 0, L.stream>>>(L.members, L.first, keep, scal);
        return hipGetLastError();
    }
    template <typename T>
    static hipError_t pick(const Launch& L, int nx, int ny, DensOp op, int var, int keep,
                           const double* scal) {
        if constexpr (has_variant(NZ))
            if (var == 1 && op == kDensInvFft) return go<T, 1>(L, nx, ny, op, keep, scal);
        if constexpr (has_zcx(NZ))
            if (var == 3 && op == kDensInvFft) return go<T, 3>(L, nx, ny, op, keep, scal);
        return go<T, 0>(L, nx, ny, op, keep, scal);
    }
    static hipError_t run(const Launch& L, int prec, int nx, int ny, DensOp op, int var,
                          int keep, const double* scal) {
        return prec ? pick<double>(L, nx, ny, op, var, keep, scal)
                    : pick<float>(L, nx, ny, op, var, keep, scal);
    }
};

hipError_t launch_z_potential_kick(const Launch& L, int prec, int nx, int ny, int nz, ZOp op,
                                   KickMode kick, int variant, bool extended) {
    return dispatch_n<ZPotKick>(nz, L, prec, nx, ny, op, kick, variant, extended);
}
hipError_t launch_z_density(const Launch& L, int prec, int nx, int ny, int nz, DensOp op,
                            int variant, int keep_member, const double* rescale) {
    if (rescale != nullptr && op != kDensDirect) return hipErrorInvalidValue;
    return dispatch_n<ZDens>(nz, L, prec, nx, ny, op, variant, keep_member, rescale);
}

}  // namespace wdm
