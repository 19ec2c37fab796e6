"""The C ABI without a GPU: every symbol the headers declare is exported, and
argument errors come back as PIC_ERR_ARG (with a message) before any launch."""
import ctypes as C
import glob
import os
import re

import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def A():
    from paper_1606_02862_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        from paper_1606_02862_amd import build
        build.build()
    _capi.load()
    return _capi


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(pic_\w+)\s*\(", text, flags=re.M))
    return names


def test_every_declared_symbol_is_exported(A):
    lib = A.load()
    names = _declared()
    assert {"pic_init", "pic_step", "pic_moments", "pic_destroy"} <= names
    for n in sorted(names):
        assert hasattr(lib, n), n
        assert n in A.SIGNATURES, f"{n} missing from the binding"


def _init(A, cfg, shape=None, nsp=None, mutate=None):
    from paper_1606_02862_amd.pic import grid_struct, species_structs
    g = grid_struct(cfg)
    s = species_structs(cfg)
    if mutate:
        mutate(g, s)
    h = C.c_void_p(123)
    shp = shape if shape is not None else {"cic": 1, "tsc": 2, "pcs": 3}[cfg["grid"]["shape"]]
    rc = A.load().pic_init(C.byref(h), C.byref(g), s, len(cfg["species"]) if nsp is None else nsp, shp, None, None)
    return rc, h, A.load().pic_last_error(None).decode()


@pytest.mark.parametrize("what,mutate,needle", [
    ("nx not a multiple of 8", lambda g, s: setattr(g, "nx", 12), "multiple"),
    ("nz not a multiple of 4", lambda g, s: setattr(g, "nz", 6), "multiple"),
    ("Courant", lambda g, s: setattr(g, "dt", 0.6), "Courant"),
    ("negative dx", lambda g, s: setattr(g, "dx", -1.0), "positive"),
    ("zero mass", lambda g, s: setattr(s[0], "mass", 0.0), "mass"),
    ("drift >= c", lambda g, s: s[0].drift_beta.__setitem__(0, 1.0), "drift_beta"),
    ("bad layout", lambda g, s: setattr(s[0], "layout", 7), "layout"),
    ("coincident with itself", lambda g, s: setattr(s[0], "coincident_with", 0), "coincident"),
    ("z_init > z_max", lambda g, s: (setattr(s[0], "z_max", 2), setattr(s[0], "z_init", 3),
                                     s[0].ionization_ev.__setitem__(0, 1.0), s[0].ionization_ev.__setitem__(1, 2.0)),
     "z_init"),
    ("ionize_into without charge states", lambda g, s: setattr(s[0], "ionize_into", 0), "ionize_into"),
    ("cap below ppc", lambda g, s: setattr(s[0], "cap_ppc", 3), "cap_ppc"),
    ("unknown gather", lambda g, s: setattr(g, "gather", 2), "gather"),
    ("unknown option", lambda g, s: setattr(g, "options", 4), "options"),
    ("deterministic J in FP64", lambda g, s: (setattr(g, "options", 1), setattr(g, "precision", 1)), "FP32"),
])
def test_init_rejects_bad_arguments(A, what, mutate, needle):
    rc, h, msg = _init(A, workloads.config(0), mutate=mutate)
    assert rc == A.PIC_ERR_ARG, what
    assert h.value is None
    assert needle in msg, msg


def _set(obj, **kw):
    for k, v in kw.items():
        setattr(obj, k, v)


@pytest.mark.parametrize("what,mutate,needle", [
    ("subshell 0 without electrons", lambda g, s: _set(s[1].lotz[2][0], q=0), "subshell 0"),
    ("subshell 0 off the ionisation energy", lambda g, s: _set(s[1].lotz[2][0], p_ev=50.0), "subshell 0"),
    ("inner subshell below the threshold", lambda g, s: _set(s[1].lotz[2][1], p_ev=10.0, a=4.5e-14, q=2), "subshell 1"),
    ("b above 1", lambda g, s: _set(s[1].lotz[0][0], b=1.5), "subshell 0"),
    ("negative c", lambda g, s: _set(s[1].lotz[0][0], c=-0.1), "subshell 0"),
    ("zero a", lambda g, s: _set(s[1].lotz[3][0], a=0.0), "subshell 0"),
    ("gap in subshells", lambda g, s: _set(s[1].lotz[1][2], p_ev=300.0, a=4.5e-14, q=2), "unused slot"),
    ("max_events", lambda g, s: _set(s[1], max_events=9), "max_events"),
    ("energy_loss", lambda g, s: _set(s[1], energy_loss=2), "energy_loss"),
])
def test_init_rejects_bad_ionisation_data(A, what, mutate, needle):
    rc, h, msg = _init(A, workloads.reduced(3, 8, 8, 4), mutate=mutate)
    assert rc == A.PIC_ERR_ARG, what
    assert h.value is None
    assert needle in msg, msg


def test_init_rejects_bad_shape_and_species_count(A):
    rc, _, msg = _init(A, workloads.config(0), shape=4)
    assert rc == A.PIC_ERR_ARG and "shape" in msg
    rc, _, msg = _init(A, workloads.config(0), nsp=0)
    assert rc == A.PIC_ERR_ARG and "n_species" in msg


def test_init_rejects_bad_precision_and_fp64_ionisation(A):
    rc, _, msg = _init(A, workloads.config(0), mutate=lambda g, s: setattr(g, "precision", 2))
    assert rc == A.PIC_ERR_ARG and "precision" in msg
    # the FP64 variant covers the PIC cycle; ionisation stays FP32
    cfg = workloads.reduced(3, 8, 8, 4)
    cfg["grid"]["precision"] = "fp64"
    rc, _, msg = _init(A, cfg)
    assert rc == A.PIC_ERR_ARG and "FP32" in msg


def test_null_handles(A):
    lib = A.load()
    assert lib.pic_step(None, 1) == A.PIC_ERR_ARG
    assert lib.pic_destroy(None) == A.PIC_OK
    assert lib.pic_abi_version() == 7
    m = A.MomentsT()
    assert lib.pic_moments(None, C.byref(m)) == A.PIC_ERR_ARG
    r = A.RunStateT()
    assert lib.pic_get_run_state(None, C.byref(r)) == A.PIC_ERR_ARG
    assert lib.pic_set_run_state(None, C.byref(r)) == A.PIC_ERR_ARG


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1606_02862_amd import _capi
    monkeypatch.setattr(_capi, "_lib", None)
    monkeypatch.setattr(_capi, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _capi.load()


def test_load_brings_in_torch_first(A):
    # torch's bundled HIP runtime and the system one share a soname, so the
    # library must be opened after torch in a fresh process; otherwise the
    # two sides bind different runtimes
    import subprocess
    import sys
    code = ("import sys; import paper_1606_02862_amd as P; assert 'torch' not in sys.modules; "
            "P.load(); assert 'torch' in sys.modules; "
            "m = [l for l in open('/proc/self/maps') if 'libamdhip64' in l]; "
            "print(len({l.split()[-1] for l in m}))")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip() == "1"  # exactly one HIP runtime mapped


def test_gauss_laguerre_rule_matches_numpy(A):
    """The library's own Golub-Welsch rule (host code) against numpy's laggauss."""
    import numpy as np
    from numpy.polynomial.laguerre import laggauss
    from paper_1606_02862_amd.pic import gauss_laguerre64
    x, w = gauss_laguerre64()
    xr, wr = laggauss(64)
    assert np.max(np.abs(x / xr - 1)) < 1e-12
    assert np.max(np.abs(w - wr)) < 1e-12          # numpy's own weights carry ~1e-13 errors
    big = wr > 1e-200
    assert np.max(np.abs(w[big] / wr[big] - 1)) < 1e-10
    # defining property of the rule: exact for polynomials up to degree 127 (checked to 20)
    import math
    for m in range(0, 21):
        assert abs(np.sum(w * x**m) / math.factorial(m) - 1.0) < 1e-14


def test_struct_layouts_match_the_header(A, tmp_path):
    """Every struct the binding declares has the size and field offsets the C
    compiler gives the header's typedef (a C program built with gcc prints
    them), so no field is read at the wrong place."""
    pairs = {"pic_grid_t": A.GridT, "pic_lotz_shell_t": A.LotzShellT, "pic_species_t": A.SpeciesT,
             "pic_alloc_t": A.AllocT, "pic_moments_t": A.MomentsT, "pic_particles_view_t": A.ParticlesViewT,
             "pic_particles64_view_t": A.ParticlesView64T, "pic_timing_t": A.TimingT,
             "pic_ionize_stats_t": A.IonizeStatsT, "pic_mlp_train_cfg_t": A.MlpTrainCfgT,
             "pic_mlp_report_t": A.MlpReportT, "pic_run_state_t": A.RunStateT}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pic.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in pairs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])
