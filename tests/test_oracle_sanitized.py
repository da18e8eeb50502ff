"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code only).

oracle.cpp is built a second time with -fsanitize=address,undefined (errors fatal) into a
temporary library, and a child process runs it through every boundary configuration of
the adjoint pins: a 3-step forward run with statistics and wall statistics, the STG plane,
one adjoint step, and a 3-step checkpoint-free gradient.  Any out-of-bounds access, use of
freed memory or undefined operation aborts the child.  The results themselves are not
checked here (the other oracle tests pin them)."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent("""
    import sys
    import numpy as np
    sys.path[:0] = [ROOT, ROOT + "/tests"]
    import oracle as O
    O._LIB = LIB
    import test_oracle_adjoint as TA
    g = np.random.default_rng(0)
    n = 0
    for name, kw in TA.CASES.items():
        cfg, f, hist, stg = TA.setup(**kw)
        open_ = cfg.xbc == 1
        planes = [1, 3]
        acc = np.zeros((2, cfg.ny, 9))
        wall = np.zeros((2, cfg.nx)) if cfg.wall_model else None
        st, f3, h3 = O.run(cfg, f, hist, 0.0, 3, stg=stg if open_ else None, planes=planes, acc=acc,
                           wall_acc=wall)
        assert st == O.OK, (name, st)
        if open_:
            assert O.stg_plane(cfg, stg, 4.0, want_fluct=True)[0] == O.OK
        lam = g.normal(size=f.shape)
        eta = g.normal(size=(5, cfg.ny, cfg.nz)) if open_ else None
        coef = g.normal(size=(2, cfg.ny, 9))
        adj = O.adjoint_step(cfg, f3, h3 if open_ else None, 4.0, lam, eta, stg=stg if open_ else None,
                             planes=planes, coef=coef, want_amp=open_)
        assert adj["status"] == O.OK, (name, adj["status"])
        if open_:
            r = O.gradient_run(cfg, stg, f, hist, 0.0, 3, planes, coef * 1e-3)
            assert np.all(np.isfinite(r["g_amp"])) and np.isfinite(r["g_cs"])
        n += 1
    print("sanitized oracle ran", n, "configurations")
""")


def _runtime(name):
    p = subprocess.run(["g++", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_oracle_runs_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if asan is None or ubsan is None:
        pytest.skip("sanitizer runtimes not installed")
    lib = str(tmp_path / "liboracle_san.so")
    src = os.path.join(ROOT, "oracle", "oracle.cpp")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", lib, src], check=True)
    env = dict(os.environ, LD_PRELOAD=asan + ":" + ubsan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="1")
    code = "ROOT = %r\nLIB = %r\n" % (ROOT, lib) + CHILD
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "sanitized oracle ran" in r.stdout
