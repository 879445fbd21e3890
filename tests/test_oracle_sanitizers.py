"""The checker under sanitizers (CPU only).

* AddressSanitizer + UndefinedBehaviorSanitizer: the oracle rebuilt with both
  (every undefined-behaviour report aborts) runs the traversal and physics pins
  in a child process with the ASan runtime preloaded; an out-of-bounds access,
  use after free or undefined operation anywhere in those paths fails the run.
* ThreadSanitizer: the oracle rebuilt with clang's TSan and LLVM's OpenMP
  runtime (its Archer tool gives TSan OpenMP's barriers) runs the OpenMP packet
  loop on four threads and must agree with one thread.
"""
import glob
import os
import subprocess
import sys

import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow


def _gcc_runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _env(**extra):
    env = dict(os.environ)
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    env.update(extra)
    return env


def test_oracle_pins_under_asan_and_ubsan():
    asan = _gcc_runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    O.build(force=True, variant="asan")
    env = _env(LD_PRELOAD=asan, QRT_ORACLE_VARIANT="asan",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-p", "no:xdist",
                        "tests/test_oracle_traversal.py", "tests/test_oracle_physics.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]


TSAN_SCRIPT = """
import numpy as np
from oracle import oracle as O
from synth import scenes
assert O.lib()._name.endswith("liboracle_tsan.so")
sc = scenes.disk128(n_packets=1 << 10, n=16).replace(max_orders=4, npix=16)
a, ca, _ = O.run(sc, O.SOBOL, 1, sc.n_packets, nthreads=4)
b, cb, _ = O.run(sc, O.SOBOL, 1, sc.n_packets, nthreads=1)
assert ca["packets"] == cb["packets"] == sc.n_packets and ca["visits"] == cb["visits"]
assert np.allclose(a, b, rtol=1e-12, atol=1e-300)
print("tsan-run-ok")
"""


def test_oracle_openmp_loop_under_tsan():
    tsan = sorted(glob.glob(os.path.join(O.LLVM_BIN, "..", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.tsan-x86_64.so")))
    archer = os.path.join(O.LLVM_BIN, "..", "lib", "libarcher.so")
    if not tsan or not os.path.exists(archer) or not os.path.exists(os.path.join(O.LLVM_BIN, "clang")):
        pytest.skip("LLVM's clang, its TSan runtime or the Archer OpenMP tool is not installed")
    O.build(force=True, variant="tsan")
    env = _env(LD_PRELOAD=tsan[-1], OMP_TOOL_LIBRARIES=archer, QRT_ORACLE_VARIANT="tsan",
               TSAN_OPTIONS="halt_on_error=1 ignore_noninstrumented_modules=1")
    r = subprocess.run([sys.executable, "-c", TSAN_SCRIPT], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    assert "tsan-run-ok" in out and "ThreadSanitizer" not in out, out[-3000:]
