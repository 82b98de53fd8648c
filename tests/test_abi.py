"""The C-ABI library on the host: it loads, exports every function include/ppcmh.h
declares, lays out its structs as the binding does, and rejects bad arguments with the
documented status before touching a device (so these run without a GPU)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from workloads import coax

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ppcmh.h")


def _lib():
    from paper_1905_13076_amd import _native
    return _native.load(), _native


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ppc_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib, nat = _lib()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
        assert n in nat.SIGNATURES, n
    out = subprocess.run(["nm", "-D", "--defined-only", nat.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ppc_\w+)", out))
    assert set(names) <= exported
    assert lib.ppc_version() == 4


def test_struct_layout_matches_binding(tmp_path):
    """sizeof/offsetof from the C compiler against the ctypes mirror."""
    _, nat = _lib()
    src = tmp_path / "probe.c"
    structs = {"ppc_mesh": nat.Mesh, "ppc_law": nat.Law, "ppc_material": nat.Material,
               "ppc_excitation": nat.Excitation, "ppc_params": nat.Params, "ppc_stats": nat.Stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    for cname, cls in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)


def _validate(prob):
    import paper_1905_13076_amd as P
    return P.validate(prob)


def _mutant(**changes):
    p = coax.c1(nr=4, ntheta=8)
    for k, v in changes.items():
        setattr(p, k, v)
    return p


def test_valid_problems_pass():
    for gen in (coax.c1, coax.c2, coax.c5_small):
        assert _validate(gen())[0] == 0


@pytest.mark.parametrize("case,code,needle", [
    ("repeat", -2, "repeats a node"),
    ("range", -2, "out-of-range"),
    ("degenerate", -2, "degenerate"),
    ("nodir", -2, "Dirichlet"),
    ("orphan", -2, "belongs to no triangle"),
    ("island", -2, "no Dirichlet node"),
    ("sigma", -1, "sigma"),
    ("matid", -1, "mat_id"),
    ("law", -1, "linear law"),
    ("brauer", -1, "Brauer"),
    ("js", -1, "js"),
    ("nh", -1, "n_h"),
    ("xy", -1, "coordinate"),
])
def test_invalid_problems_are_rejected_on_host(case, code, needle):
    p = _mutant()
    if case == "repeat":
        p.tri = p.tri.copy(); p.tri[3] = [p.tri[3][0], p.tri[3][0], p.tri[3][2]]
    elif case == "range":
        p.tri = p.tri.copy(); p.tri[2, 1] = p.n_nodes
    elif case == "degenerate":
        p.xy = p.xy.copy(); a, b, c = p.tri[10]; p.xy[c] = 0.5 * (p.xy[a] + p.xy[b])
    elif case == "nodir":
        p.dirichlet = np.zeros(0, np.int32)
    elif case == "orphan":
        p.xy = np.vstack([p.xy, [[1.0, 1.0]]])
    elif case == "island":
        extra = np.array([[1.0, 1.0], [1.1, 1.0], [1.0, 1.1]])
        n0 = p.n_nodes
        p.xy = np.vstack([p.xy, extra])
        p.tri = np.vstack([p.tri, [[n0, n0 + 1, n0 + 2]]]).astype(np.int32)
        for f in ("sigma", "js"):
            setattr(p, f, np.append(getattr(p, f), 0.0))
        p.mat_id = np.append(p.mat_id, 0).astype(np.int32)
    elif case == "sigma":
        p.sigma = p.sigma.copy(); p.sigma[0] = -1.0
    elif case == "matid":
        p.mat_id = p.mat_id.copy(); p.mat_id[0] = 5
    elif case == "law":
        p.mat_par = np.array([[0.0, 0, 0, 0]])
    elif case == "brauer":
        p.mat_model = np.array([1]); p.mat_par = np.array([[0.0, 3.8, 2.17, 0.0]])
    elif case == "js":
        p.js = p.js.copy(); p.js[4] = np.nan
    elif case == "nh":
        p.orders = np.arange(17); p.amps = np.ones(17); p.phases = np.zeros(17)
    elif case == "xy":
        p.xy = p.xy.copy(); p.xy[3, 0] = np.inf
    rc, msg = _validate(p)
    assert rc == code and needle in msg, (rc, msg)


@pytest.mark.parametrize("kw,needle", [
    (dict(N=3), "even"), (dict(N=0), "even"), (dict(m=0), "m must"), (dict(T=-1.0), "T must"),
    (dict(tol_lin=1.5), "tol_lin"), (dict(shift_mode=2), "shift_mode"), (dict(precision=7), "precision"),
    (dict(block=100), "block"), (dict(max_newton=0), "max_newton"), (dict(tol_ppc=float("nan")), "tol_ppc"),
    (dict(coarse_precision=2), "coarse_precision"), (dict(coarse_precision=-2), "coarse_precision"),
    (dict(graph=2), "graph"), (dict(b_cap=-1.0), "b_cap"), (dict(b_cap=float("inf")), "b_cap"),
    (dict(init_mode=5), "init_mode"), (dict(method=2), "method"), (dict(method=-1), "method"),
    (dict(method=1, b_cap=3.0), "b_cap"), (dict(fine_block=128), "fine_block"),
    (dict(fine_block=512, block=1024), "fine_block"), (dict(n_harm=7), "n_harm"),
    (dict(n_harm=-1), "n_harm"), (dict(method=1, n_harm=3), "n_harm"),
    (dict(coarse_mode=2), "coarse_mode"), (dict(coarse_mode=-1), "coarse_mode"),
    (dict(coarse_mode=1, method=1), "coarse_mode"), (dict(coarse_mode=1, n_harm=3), "coarse_mode"),
    (dict(coarse_mode=1, b_cap=3.0), "coarse_mode"),
    (dict(lin_start=3), "lin_start"), (dict(lin_start=-1), "lin_start"),
    (dict(lin_forcing=2), "lin_forcing"),
    (dict(tol_adapt=-1e-3), "tol_adapt"), (dict(tol_adapt=1.0), "tol_adapt"),
])
def test_invalid_params_are_rejected_on_host(kw, needle):
    import paper_1905_13076_amd as P
    rc, msg = P.validate_params(P.params(**kw))
    assert rc == -1 and needle in msg, (rc, msg)
    assert P.validate_params(P.params())[0] == 0


def test_null_safety_and_no_device_error():
    lib, nat = _lib()
    assert lib.ppc_destroy(None) == 0
    assert lib.ppc_problem_destroy(None) == 0
    assert lib.ppc_params_default(None) == -1
    assert lib.ppc_problem_info(None, None, None, None, None) == -1
    assert lib.ppc_fine_counts(None, 4, None) == -1
    assert lib.ppc_autotune(None, None, None, None, None) == -1
    assert lib.ppc_time_stepping_device(None, None, None, None, None, None, None, None, None) == -1
    assert lib.ppc_last_error(None) is not None
    h = ctypes.c_void_p()
    assert lib.ppc_create(-1, ctypes.byref(h)) == -1
    assert lib.ppc_problem_create(None, None, None, None, ctypes.byref(h)) == -1
    import torch
    if not torch.cuda.is_available():
        rc = lib.ppc_create(0, ctypes.byref(h))
        assert rc == -3 and not h.value
        assert b"GPU" in lib.ppc_last_error(None)
