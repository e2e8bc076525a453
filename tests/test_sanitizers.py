"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the CPU oracle
(gcc) and of the host lane simulator (g++, the transport kernels' per-lane
logic), driven through their usual Python wrappers in a child process with
the ASan runtime preloaded.  Every scenario runs to completion without a
sanitizer report: Cartesian and octree grids, point / anisotropic /
exponential-disk / dust sources, second moments, histories, the learned
proposal, dust emission, event caps and tau cuts, degenerate media."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1",
       "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]

DRIVER = textwrap.dedent("""
    import numpy as np
    import oracle, lanesim
    from paper_1705_04702_amd import scenes
    theta = scenes.init_mlp(3, scale=1.5).astype(np.float32)
    cases = [
        scenes.sphere(n=8, tau=1.0, albedo=0.5, g=0.5, npix=16),
        scenes.uniform_cube(2, 2.0, 0.7, 0.8, src=(0.3, -0.9, 0.99)),
        scenes.disk((12, 10, 6), 3, 16),
        scenes.torus(5, 4, 3, 16, n_clumps=12, tau_eq=6.0),
    ]
    capped = scenes.sphere(n=6, tau=4.0, albedo=0.95)
    capped.event_cap = 2
    cut = scenes.disk((8, 8, 4), 2, 8, tau_v_faceon=4.0)
    cut.tau_peel_max = 1.0
    empty = scenes.sphere(n=4)
    empty.density[:] = 0.0
    outside = scenes.uniform_cube(2, 1.0, 0.6, 0.2, src=(3.0, 0.2, -0.1))
    outside.instruments = []
    cases += [capped, cut, empty, outside]
    for sc in cases:
        oracle.run(sc, 60, seed=1, moments=True)
        oracle.run(sc, 60, seed=2, first_id=7, count=31, histories=4)
        for prec in (0, 1):
            lanesim.run(sc, 40, seed=3, precision=prec)
        oracle.run(sc, 30, seed=4, mlp=theta)
        lanesim.run(sc, 20, seed=4, precision=1, mlp=theta)
        lanesim.run(sc, 20, seed=5, precision=0, histories=3)
    for sc in (cases[0], cases[3]):
        r = oracle.run(sc, 80, seed=6)
        T, em = oracle.dust_emission(sc, r["table"])
        oracle.run(oracle.dust_scene(sc, em), 40, seed=7)
    print("sanitized runs ok", flush=True)
""")


def _lib(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if out and os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.timeout(600)
def test_oracle_and_lane_simulator_under_asan_ubsan(tmp_path):
    asan = _lib("libasan.so")
    if asan is None or _lib("libubsan.so") is None:
        pytest.skip("gcc sanitizer runtimes not installed")
    o_lib = str(tmp_path / "oracle_san.so")
    l_lib = str(tmp_path / "lanesim_san.so")
    subprocess.check_call(["gcc", "-std=c11", *SAN, "-o", o_lib, os.path.join(ROOT, "oracle", "mcrt_oracle.c"),
                           "-lm"])
    csrc = os.path.join(ROOT, "paper_1705_04702_amd", "csrc")
    subprocess.check_call(["g++", "-std=c++17", *SAN, f"-I{csrc}", "-o", l_lib, os.path.join(csrc, "lanesim.cpp")])
    env = dict(os.environ)
    env.update(LD_PRELOAD=asan, MCRT_ORACLE_LIB=o_lib, MCRT_LANESIM_LIB=l_lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               PYTHONPATH=os.pathsep.join([ROOT, os.path.join(ROOT, "tests"), env.get("PYTHONPATH", "")]))
    r = subprocess.run([sys.executable, "-c", DRIVER], env=env, capture_output=True, text=True, timeout=550)
    report = r.stdout[-3000:] + r.stderr[-6000:]
    assert r.returncode == 0, report
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, report
    assert "sanitized runs ok" in r.stdout
