"""Host sanitizer runs (CPU only).

The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc) runs noise, rollout (every cost term, null particles), update, the
gradient, the ball model and the learned self-collision network on small
inputs; the C-ABI library built with its host code instrumented by
AddressSanitizer (clang, through hipcc; the gfx950 device code is built as
usual) runs the ABI validation tests.  Each run is a child process with the
sanitizer runtime preloaded; any report fails the test."""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

ORACLE_CALLS = """
import numpy as np, oracle
from paper_2104_13542_amd import inputs
p = inputs.config2(3, n_particles=12, horizon=8, n_obs_spheres=3, n_obs_cuboids=3)
p.params.n_null = 2
o = oracle.Oracle(p)
eps = o.noise(1)
ro = o.rollout(np.zeros((8, 7)), np.full(7, 0.3), eps)
up = o.update(ro["C"], ro["u"], np.zeros((8, 7)), np.full(7, 0.09))
p.params.cov_per_step = 1
o2 = oracle.Oracle(p)
up2 = o2.update(ro["C"], ro["u"], np.zeros((8, 7)), np.full((8, 7), 0.09))
p4 = inputs.config4(2)
p4.params.n_particles, p4.params.horizon, p4.params.dt = 9, 6, np.full(6, 0.02)
o4 = oracle.Oracle(p4)
g, J = o4.grad(np.zeros((6, 7)), np.full(7, 0.1), o4.noise(0))
ec = o4.expected_cost(np.zeros((6, 7)), np.full(7, 0.1), o4.noise(0))
pb = inputs.config_ball(1, n_particles=6, horizon=5)
ob = oracle.Oracle(pb)
ob.set_ball(ob.ball_world_from_tray(pb.ball_tray))
rb = ob.rollout(np.zeros((5, 7)), np.full(7, 0.3), ob.noise(0))
ps = inputs.config_self_mlp(1, n_particles=5, horizon=4)
on = oracle.Oracle(ps)
rn = on.rollout(np.zeros((4, 7)), np.full(7, 0.3), on.noise(0))
fr = oracle.fk(o.dh, np.zeros(7))
m = oracle.manipulability(oracle.jacobian(fr))
xd, xdd = oracle.task_space(o.dh, np.full(7, 0.2), np.full(7, 0.1), np.full(7, 0.05))
assert np.all(np.isfinite(ro["C"])) and np.isfinite(J) and np.isfinite(m)
print("SANITIZED RUN OK")
"""


def _run(code, env):
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=900, cwd=ROOT)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    return r.stdout


def test_oracle_under_asan_and_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_sanitized.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
                           os.path.join(ROOT, "oracle", "storm_oracle.c"), "-o", lib, "-lm"])
    rt = " ".join(subprocess.check_output(["gcc", "-print-file-name=" + n]).decode().strip()
                  for n in ("libasan.so", "libubsan.so"))
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    code = "import sys; sys.path.insert(0, %r)\nimport oracle\noracle._LIB = %r\n" % (ROOT, lib) + \
        textwrap.dedent(ORACLE_CALLS)
    assert "SANITIZED RUN OK" in _run(code, env)


def test_abi_validation_under_asan(tmp_path):
    rts = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rts:
        pytest.skip("clang AddressSanitizer runtime not found")
    sys.path.insert(0, ROOT)
    from paper_2104_13542_amd import build

    lib = str(tmp_path / "libstorm_host_asan.so")
    flags = [f for f in build.HIPCC_FLAGS if f != "-O3"] + ["-O1", "-g", "-Xarch_host", "-fsanitize=address",
                                                            "-Xarch_host", "-fno-omit-frame-pointer"]
    subprocess.check_call([os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), *flags, "-I", os.path.join(ROOT, "include"),
                           "-I", build.CSRC, *build.sources(), "-o", lib], stderr=subprocess.DEVNULL)
    env = dict(os.environ, LD_PRELOAD=rts[0], ASAN_OPTIONS="detect_leaks=0")
    code = textwrap.dedent("""
        import sys
        sys.path.insert(0, %r)
        import paper_2104_13542_amd.storm as s
        s.LIB_PATH = %r
        assert s.lib()._name == %r
        import pytest
        rc = pytest.main(["-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu", %r])
        print("ABI VALIDATION RC", int(rc))
        sys.exit(int(rc))
    """) % (ROOT, lib, lib, os.path.join(ROOT, "tests", "test_abi.py"))
    assert "ABI VALIDATION RC 0" in _run(code, env)
