"""Host code under the sanitizers (CPU only).

- The FP64 oracle (plain C) built with AddressSanitizer and
  UndefinedBehaviorSanitizer (gcc), driven through every C entry point:
  whole cycles of each shape and gather, the threaded cycle, the
  diagnostics, and the single routines on particles near the periodic seams.
- The library's host code (the C ABI, its argument checks and set-up, the
  Gauss-Laguerre rule) built with AddressSanitizer for the host pass only,
  running the ABI tests; the host build of the particle kernel's deposit
  arithmetic running its tests the same way.
- A copy of the oracle with an out-of-bounds read planted in it fails the
  sanitized run, so the runs above would have caught one.

Each run is a child process with the sanitizer runtime preloaded (the Python
interpreter itself is not instrumented).
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "paper_1606_02862_amd", "_build")
CSRC = os.path.join(ROOT, "paper_1606_02862_amd", "csrc")

pytestmark = pytest.mark.slow

# gcc builds of the oracle: IEEE FP64 as in its default build, plus the checks
ORACLE_SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=all"]
# host pass only: the device code of the same sources is compiled as usual
HOST_ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
ASAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
            "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}

ORACLE_DRIVER = r"""
import sys
import oracle, workloads
oracle.use_library(oracle.load_library(sys.argv[1]))
cases = [(0, (16, 16, 16), "cic", "standard"), (1, (16, 16, 8), "cic", "galerkin"),
         (2, (16, 16, 8), "tsc", "galerkin"), (0, (16, 16, 8), "pcs", "standard"),
         (5, (16, 16, 8), "tsc", "standard"), (3, (16, 16, 8), "tsc", "standard")]
for idx, box, shape, gather in cases:
    cfg = workloads.config(idx, nx=box[0], ny=box[1], nz=box[2], shape=shape, gather=gather)
    st = oracle.init_state(cfg)
    oracle.energy_trace_total(oracle.step(st, 2, trace=True))
    oracle.step_threads(st, 1, 4)
    oracle.gauss_residual(st)
    oracle.kinetic(st)
    g = st.grid
    oracle.div_cells(g, st.B)
    oracle.field_energy(g, st.E, st.B)
    s = st.species[0]
    # particles at the upper seams, moved across them
    n = 64
    x = g.nx - 0.25 + 0.0 * s.x[:n]
    y = g.ny - 1e-9 + 0.0 * s.y[:n]
    z = s.z[:n]
    Ep, Bp = oracle.gather(g, st.E, st.B, x, y, z)
    oracle.boris(-1.0, 0.5, Ep, Bp, s.ux[:n], s.uy[:n], s.uz[:n])
    oracle.esirkepov(g, s.w[:n], x, y, z, (x + 0.4) % g.nx, (y + 0.3) % g.ny, z)
    oracle.deposit_rho(g, s.w[:n], x, y, z)
oracle.philox4x64_10([1, 2, 3, 4], [5, 6])
oracle.u01(12345)
for order in (1, 2, 3):
    oracle.shape(order, 0.3)
print("oracle driver done", flush=True)
"""


def _runtime_gcc():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _runtime_clang():
    r = subprocess.run(["hipcc", "--print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    p = r.stdout.strip().splitlines()[-1] if r.returncode == 0 and r.stdout.strip() else ""
    if os.path.isabs(p) and os.path.exists(p):
        return p
    r = subprocess.run(["hipcc", "--print-resource-dir"], capture_output=True, text=True)
    p = os.path.join(r.stdout.strip().splitlines()[-1], "lib", "linux", "libclang_rt.asan-x86_64.so") \
        if r.returncode == 0 and r.stdout.strip() else ""
    return p if os.path.exists(p) else None


def _run(cmd, runtime, extra_env=None, timeout=600):
    env = dict(os.environ, **ASAN_ENV, LD_PRELOAD=runtime, PYTHONPATH=ROOT)
    env.update(extra_env or {})
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)


def _build_oracle(src, out):
    subprocess.check_call(["gcc", *ORACLE_SAN, "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                           "-fopenmp", "-shared", "-o", out, src, "-lm"])
    return out


@pytest.fixture(scope="module")
def gcc_rt():
    rt = _runtime_gcc()
    if rt is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    return rt


def test_oracle_under_address_and_undefined_sanitizers(tmp_path, gcc_rt):
    so = _build_oracle(os.path.join(ROOT, "oracle", "pic_oracle.c"), str(tmp_path / "liboracle_san.so"))
    r = _run([sys.executable, "-c", ORACLE_DRIVER, so], gcc_rt)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "oracle driver done" in r.stdout
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]


def test_sanitized_oracle_run_catches_a_planted_overflow(tmp_path, gcc_rt):
    """The kinetic-energy sum reads one particle past the end in this copy."""
    src = open(os.path.join(ROOT, "oracle", "pic_oracle.c")).read()
    head = src.index("double orc_kinetic(")
    body_end = src.index("\n}", head)
    body = src[head:body_end]
    assert body.count("p < s->n") == 1, "the planted change no longer applies"
    planted = src[:head] + body.replace("p < s->n", "p <= s->n") + src[body_end:]
    bad = tmp_path / "pic_oracle_planted.c"
    bad.write_text(planted)
    so = _build_oracle(str(bad), str(tmp_path / "liboracle_planted.so"))
    script = ("import sys, oracle, workloads\n"
              "oracle.use_library(oracle.load_library(sys.argv[1]))\n"
              "st = oracle.init_state(workloads.config(0, nx=8, ny=8, nz=4))\n"
              "print(oracle.kinetic(st))\n")
    r = _run([sys.executable, "-c", script, so], gcc_rt)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr, r.stderr[-3000:]


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_library_host_code_under_address_sanitizer(tmp_path):
    rt = _runtime_clang()
    if rt is None:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    host_srcs = ("pic_api.hip", "quadrature.hip")
    others = sorted(os.path.join(BUILD, f) for f in os.listdir(BUILD)
                    if f.endswith(".o") and f[:-2] + ".hip" not in host_srcs) if os.path.isdir(BUILD) else []
    expected = sorted(f[:-4] for f in os.listdir(CSRC) if f.endswith(".hip") and f not in host_srcs)
    if [os.path.basename(o)[:-2] for o in others] != expected:
        pytest.skip("the library's objects are not built (paper_1606_02862_amd.build.build())")
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-munsafe-fp-atomics",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-function"]
    objs = []
    for f in host_srcs:
        o = str(tmp_path / (f[:-4] + ".o"))
        r = subprocess.run(["hipcc", *flags, *HOST_ASAN, "-c", os.path.join(CSRC, f), "-o", o],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(o)
    lib = str(tmp_path / "libpic_asan.so")
    r = subprocess.run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib, *others, *objs],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    nm = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in nm, "the host pass is not instrumented"
    from tests import host
    dep = host.build(so=str(tmp_path / "libdeposit_asan.so"), extra=tuple(HOST_ASAN), force=True)
    r = _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-p", "tests.host.asan_plugin",
              "tests/test_abi.py", "tests/test_deposit_host.py"], rt,
             {"PIC_ASAN_LIB": lib, "PIC_ASAN_DEPOSIT": dep})
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out, out[-4000:]
    assert " passed" in r.stdout and "failed" not in r.stdout and "error" not in r.stdout, r.stdout[-2000:]
