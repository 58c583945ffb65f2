"""Write sampled FP64-oracle results for the precision study's 128^3 sub-box.

Workload: the GRF + soliton generator (k0 = 16 * 2 pi absolute, rho_c = 50,
r_c = 0.03, seed 0) on a box of L' = 0.25 with 128^3 nodes -- the same dx = 1/512
and dt = 0.2 dx^2 as the 512^3 run it samples -- no particles.  The oracle runs
`steps` unmerged KDK steps; the file keeps psi at 65536 seeded random cells,
the total mass and the oracle's energy before and after.  Values come from
oracle/ and the seeded input generator only.

    python tests/golden/make_subbox_reference.py [steps]
"""
import math
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import oracle  # noqa: E402
from paper_2606_25026_amd import inputs  # noqa: E402

N, L, SEED = 128, 0.25, 0


def subbox_field():
    return inputs.grf_soliton(N, L=L, k0=16.0 * 2 * math.pi, rc=0.03, rho_c=50.0, seed=SEED)


def main(steps: int = 2000) -> Path:
    oracle.set_threads(0)
    psi0 = subbox_field()
    dx = L / N
    dt = 0.2 * dx * dx
    cfg = oracle.make_config((N,) * 3, L=L)
    e0 = oracle.energy(cfg, psi0)
    t0 = time.time()
    psi, _, _ = oracle.kdk(cfg, psi0, nsteps=steps, dt=dt)
    elapsed = time.time() - t0
    e1 = oracle.energy(cfg, psi)
    rng = np.random.default_rng(54321)
    cells = np.sort(rng.choice(N ** 3, size=65536, replace=False))
    out = Path(__file__).resolve().parent / f"subbox_128_steps{steps}.npz"
    np.savez_compressed(out, cells=cells, psi=psi.ravel()[cells], psi0=psi0.ravel()[cells],
                        steps=steps, dt=dt, n=N, L=L, seed=SEED, mass0=e0["mass"],
                        mass1=e1["mass"], etot0=e0["e_total"], etot1=e1["e_total"],
                        oracle_seconds=elapsed, oracle_threads=oracle.get_threads())
    print(f"wrote {out} ({steps} steps in {elapsed:.1f} s on {oracle.get_threads()} threads)")
    return out


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 2000)
