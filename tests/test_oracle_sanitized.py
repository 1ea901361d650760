"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): the oracle library is rebuilt with both sanitizers into a
temporary directory and a child process steps small mechanics, cell
behaviour, SIR and diffusion cases through it; any out-of-bounds access,
use after free or undefined operation aborts the child."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import sys
import numpy as np
sys.path.insert(0, ROOT)
from oracle import sim as osim
osim._LIB_PATH = LIB
from oracle import sir as osir
from oracle import soma as osoma
from paper_2503_10796_amd import inputs

pos, diam = inputs.plain(300, 60.0, seed=0)
o = osim.OracleSim(pos, diam, osim.make_params(box_len=15.0, detect_static=True))
o.step(3)
vdiv = inputs.division_volume(9.0)
pos, diam, vol, growth = inputs.spheroid(200, seed=3, growth_mean=40.0)
age = np.arange(200, dtype=np.int32) % 100
o = osim.OracleSim(pos, diam, osim.make_params(box_len=0.0, div_vol=vdiv, seed=2, brownian_rate=0.01,
                                               death_prob=0.2, min_age=20, division_prob=0.5),
                   vol=vol, growth=growth, cap=2000, age=age)
o.step(5)
spos, sst = inputs.sir_population(300, 30, 30.0, seed=1)
for b in (osir.TOROIDAL, osir.CLOSED):
    osir.OracleSIR(spos, sst, osir.make_params(30.0, 3.0, 0.5, 0.05, 4.0, boundary=b, seed=1)).step(5)
cpos = np.random.default_rng(2).uniform(0, 20.0, size=(200, 3))
osoma.OracleSoma(cpos, (np.arange(200) % 2).astype(np.int32), osoma.make_params(space=20.0, resolution=9)).step(4)
print("sanitized oracle ok", flush=True)
'''


def _runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.timeout(300)
def test_oracle_is_clean_under_address_and_undefined_behaviour_sanitizers():
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no libasan for gcc on this host")
    srcs = [os.path.join(ROOT, "oracle", f) for f in ("abm_oracle.c", "sir_oracle.c", "soma_oracle.c")]
    with tempfile.TemporaryDirectory() as tmp:
        lib = os.path.join(tmp, "liboracle_san.so")
        sanitize = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer"]
        subprocess.run(["gcc", "-std=gnu11", "-O1", "-g", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                        *sanitize, *srcs, "-o", lib, "-lquadmath", "-lm"], check=True)
        env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
        code = f"ROOT = {ROOT!r}\nLIB = {lib!r}\n" + CHILD
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=280)
        assert r.returncode == 0, r.stderr[-3000:]
        assert "sanitized oracle ok" in r.stdout
