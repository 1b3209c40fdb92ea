"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle (oracle/oracle.c) and the library's host-only ray geometry
(csrc/lrt_geom.cpp: Gauss-Legendre nodes, the axisymmetric traversal, the
Fibonacci-sphere rule) are built with -fsanitize=address,undefined into a
temporary directory and exercised in child processes that preload the
sanitizer runtimes: the oracle's pins run against the instrumented oracle,
and the instrumented geometry traces the rays of the geometry tests and is
compared with the oracle's crossings.  Any report ends the child with an
error, which fails the test."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
       "-shared", "-fPIC"]


def _runtime(name):
    try:
        p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True,
                           check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.fixture(scope="module")
def san_env(tmp_path_factory):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (shutil.which("gcc") and shutil.which("g++") and asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not available")
    d = tmp_path_factory.mktemp("san")
    orc = str(d / "liboracle_san.so")
    geo = str(d / "libgeom_san.so")
    subprocess.run(["gcc", *SAN, "-fopenmp", "-ffp-contract=off", "-o", orc,
                    os.path.join(ROOT, "oracle", "oracle.c"), "-lm"], check=True)
    subprocess.run(["g++", "-std=c++17", *SAN, "-ffp-contract=off", "-o", geo,
                    os.path.join(ROOT, "paper_2604_11856_amd", "csrc", "lrt_geom.cpp")], check=True)
    env = dict(os.environ, ORACLE_LIB=orc, LD_PRELOAD=asan + ":" + ubsan,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", PYTHONPATH=ROOT, OMP_NUM_THREADS="4")
    return env, geo


def test_oracle_pins_under_sanitizers(san_env):
    env, _ = san_env
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_cr_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, tail


def test_host_geometry_under_sanitizers(san_env):
    env, geo = san_env
    script = textwrap.dedent('''
        import ctypes as C, math, sys
        import numpy as np
        import oracle as O
        from paper_2604_11856_amd import synth
        L = C.CDLL(%r)
        dp, i32p, i64p = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        L.lrt_trace_axi_ray.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                        C.c_double, C.c_int64, i32p, dp, i64p]
        L.lrt_fibonacci_quadrature.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int64, dp, dp, i64p]
        n_cases = 0
        for nx, nr, Lx, R in ((16, 20, 1.0, 0.3), (64, 32, 10.0, 8.0), (256, 128, 100.0, 50.0), (5, 7, 1.0, 1.0)):
            g = synth.AxiGeometry(nx, nr, Lx, R, np.arange(nr) * R / nr, 4, 4)
            for rw in list(g.wall_r[::max(1, nr // 6)]) + [0.0, 0.999 * R]:
                for mu in (0.05, 0.3, 0.7, 0.95, 1.0):
                    for phi in (0.0, 0.2, math.pi / 2, 2.9, math.pi, 5.5):
                        cap = nx + 2 * nr + 8
                        cell = np.zeros(cap, np.int32); ds = np.zeros(cap); n = C.c_int64()
                        s = L.lrt_trace_axi_ray(nx, nr, Lx, R, float(rw), mu, phi, cap,
                                                cell.ctypes.data_as(i32p), ds.ctypes.data_as(dp), C.byref(n))
                        assert s == 0, (nx, rw, mu, phi)
                        c2, d2 = O.axi_ray(g, float(rw), mu, phi)
                        assert abs(ds[:n.value].sum() - d2.sum()) <= 1e-12 * d2.sum()
                        n_cases += 1
                        # capacity too small and invalid directions are errors, not overruns
                        if n.value > 1:
                            assert L.lrt_trace_axi_ray(nx, nr, Lx, R, float(rw), mu, phi, n.value - 1,
                                                       cell.ctypes.data_as(i32p), ds.ctypes.data_as(dp),
                                                       C.byref(n)) != 0
                        assert L.lrt_trace_axi_ray(nx, nr, Lx, R, float(rw), 0.0, phi, cap,
                                                   cell.ctypes.data_as(i32p), ds.ctypes.data_as(dp),
                                                   C.byref(n)) != 0
        for n_los, p, a in ((400, 20, 40), (7, 3, 5), (1600, 32, 64)):
            m = C.c_int64()
            assert L.lrt_fibonacci_quadrature(n_los, p, a, 0, None, None, C.byref(m)) != 0
            dirs = np.zeros(3 * m.value); w = np.zeros(m.value)
            assert L.lrt_fibonacci_quadrature(n_los, p, a, m.value, dirs.ctypes.data_as(dp),
                                              w.ctypes.data_as(dp), C.byref(m)) == 0
            assert abs(w.sum() - math.pi) <= 1e-12
        print("geometry cases", n_cases)
    ''' % geo)
    r = subprocess.run([sys.executable, "-c", script], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
