"""The oracle's pins again, against a build with AddressSanitizer and
UndefinedBehaviorSanitizer (g++ -fsanitize=address,undefined, halting on the
first report), in a child process with the ASan runtime preloaded: an
out-of-bounds access, a use after free or undefined behaviour anywhere the pins
reach fails here even where it happens not to change a result."""
import os
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent


def runtime(name):
    r = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if r.returncode == 0 and os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.timeout(900)
def test_oracle_pins_under_asan_and_ubsan():
    asan = runtime("libasan.so")
    if asan is None:
        pytest.skip("no libasan for g++ here")
    sys.path.insert(0, str(ROOT))
    import oracle
    lib = oracle.build(sanitize=True)
    env = dict(os.environ, LD_PRELOAD=asan, ORACLE_LIB=str(lib),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    files = ["tests/test_oracle_pins.py", "tests/test_oracle_pins_nbody.py",
             "tests/test_oracle_pins_absorb_si.py", "tests/test_oracle_pins_isolated_tidal.py",
             "tests/test_oracle_pins_diagnostics.py"]
    # the five longest convergence studies repeat code paths the other pins
    # reach (the step, Poisson, the isolated step), and take 2.5 of the 3.5
    # minutes under the sanitizers
    slow = ("test_trap_ground_state_is_stationary or test_linear_jeans_growth_rate or "
            "test_second_order_convergence or test_linear_jeans_oscillation_frequency or "
            "test_isolated_steps_unitary_reversible_second_order")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", "-k", f"not ({slow})", *files], cwd=ROOT, env=env,
                       capture_output=True, text=True)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
