"""C-ABI contract checks that need no GPU.

The library loads, exports every function declared in include/fld.h, and
its host-side validation rejects bad parameters before touching a device.
"""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2503_02764_amd import fld

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fld\w*)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = fld.load()
    names = _declared("fld.h")
    assert "fld_step" in names and "fld_exchange" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(fld.EXPORTED) == sorted(names)


def test_library_exports_every_network_symbol():
    lib = fld.load()
    names = _declared("fldnn.h")
    assert "fldnn_train_step" in names and "fld_set_model" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(fld.EXPORTED_NN) == sorted(names)


def test_network_parameter_count_matches_oracle_architecture():
    from oracle import unet_ref
    n = sum(k * k * ci * co + co for _, ci, co, k in unet_ref.LAYERS)
    assert fld.fldnn_param_count() == n
    assert fld.fldnn_workspace_bytes(1, 12, 16, 0) == 0  # H not /8
    assert fld.fldnn_workspace_bytes(2, 16, 16, 1) > \
        fld.fldnn_workspace_bytes(2, 16, 16, 0) > 0


def _c_layout(struct, fields, tmp_path):
    """sizeof/offsetof of a header struct, as the C compiler lays it out."""
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fld.h"',
             "int main(void) {",
             f'  printf("%zu\\n", sizeof({struct}));']
    for f in fields:
        lines.append(f'  printf("%zu\\n", offsetof({struct}, {f}));')
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True,
                         text=True).stdout.split()
    return [int(v) for v in out]


@pytest.mark.parametrize("cls,struct", [(fld.fld_params, "fld_params"),
                                        (fld.fld_stats, "fld_stats")])
def test_struct_layout_matches_header(cls, struct, tmp_path):
    names = [n for n, _ in cls._fields_]
    got = _c_layout(struct, names, tmp_path)
    assert got[0] == ctypes.sizeof(cls)
    for name, off in zip(names, got[1:]):
        assert getattr(cls, name).offset == off, name


def test_defaults_and_workspace():
    p = fld.fld_params_default()
    assert p.ndim == 1 and p.rtol == 1e-8 and p.max_cycles == 50
    assert p.pre_smooth == 2 and p.post_smooth == 2
    p = fld.fld_params_default(ndim=2, n=(1024, 1024, 1),
                               dx=(1 / 1024, 1 / 1024, 1),
                               bc_lo=(1, 1, 1), bc_hi=(1, 1, 1))
    ws = fld.fld_workspace_bytes(p)
    # level 0: two face arrays, the rhs copy and the second iterate buffer
    # of the tiled smoother (4 x 8 MiB); the coarse levels add a third of
    # that (x, b, two faces, second buffer): about 5.7 x 8 MiB in all
    assert 4 * 8 * 2 ** 20 < ws < 6 * 8 * 2 ** 20


@pytest.mark.parametrize("field,value", [
    ("ndim", 0), ("ndim", 4), ("c", 0.0), ("a_rad", -1.0), ("gamma", 1.0),
    ("gas_const", 0.0), ("rtol", 0.0), ("rtol", 1.5), ("max_cycles", 0),
    ("limiter", 7), ("face_mean", 3), ("precision", 9), ("guess", 9),
    ("ir_inner", -1), ("ir_inner", 9), ("coarse_pre_smooth", -1),
    ("coarse_post_smooth", 17),
])
def test_invalid_params_rejected_on_host(field, value):
    p = fld.fld_params_default(ndim=1, n=(64, 1, 1), dx=(1 / 64, 1, 1))
    setattr(p, field, value)
    assert fld.fld_workspace_bytes(p) == 0
    lib = fld.load()
    out = ctypes.c_void_p()
    st = lib.fld_setup(ctypes.byref(p), ctypes.c_void_p(256), 1 << 30, None,
                       ctypes.byref(out))
    assert st == fld.FLD_ERR_INVALID_ARG
    assert lib.fld_last_error(None).decode()


def test_bc_and_shape_validation():
    lib = fld.load()
    out = ctypes.c_void_p()
    bad = [
        dict(ndim=1, n=(8, 1, 1), bc_lo=(0, 0, 0), bc_hi=(1, 0, 0)),  # half-periodic
        dict(ndim=1, n=(1, 1, 1), bc_lo=(1, 0, 0), bc_hi=(1, 0, 0)),  # 1-cell wall
        dict(ndim=1, n=(8, 2, 1)),  # unused side != 1
        dict(ndim=2, n=(8, 8, 1), dx=(0.1, -1, 1)),
        dict(ndim=1, n=(64, 1, 1), guess=fld.FLD_GUESS_LEARNED),
        dict(ndim=2, n=(64, 60, 1), guess=fld.FLD_GUESS_LEARNED),  # 60 % 8
    ]
    for kw in bad:
        p = fld.fld_params_default(**kw)
        st = lib.fld_setup(ctypes.byref(p), ctypes.c_void_p(256), 1 << 30,
                           None, ctypes.byref(out))
        assert st == fld.FLD_ERR_INVALID_ARG, kw
    # workspace checks come after parameter checks
    p = fld.fld_params_default(ndim=1, n=(64, 1, 1), dx=(1 / 64, 1, 1))
    assert lib.fld_setup(ctypes.byref(p), None, 1 << 30, None,
                         ctypes.byref(out)) == fld.FLD_ERR_WORKSPACE
    assert lib.fld_setup(ctypes.byref(p), ctypes.c_void_p(256 + 8), 1 << 30,
                         None, ctypes.byref(out)) == fld.FLD_ERR_WORKSPACE
    assert lib.fld_setup(ctypes.byref(p), ctypes.c_void_p(256), 16, None,
                         ctypes.byref(out)) == fld.FLD_ERR_WORKSPACE


def test_dirichlet_validation():
    """Dirichlet walls (FLD_BC_DIRICHLET): a positive finite wall value, a
    non-periodic dimension, and an FP64 V-cycle solve (no FP32 refinement,
    flexible CG or learned guess); a valid set-up sizes its workspace with
    the walls' diagonal terms."""
    from paper_2503_02764_amd.solver import make_params
    lib = fld.load()
    out = ctypes.c_void_p()
    D = fld.FLD_BC_DIRICHLET
    good = dict(ndim=1, n=(64, 1, 1), dx=(1 / 64, 1, 1), bc_lo=(1, 0, 0),
                bc_hi=(D, 0, 0), bc_value_hi=(2.0, 0, 0))
    p = fld.fld_params_default(**good)
    with_walls = fld.fld_workspace_bytes(p)
    p0 = fld.fld_params_default(ndim=1, n=(64, 1, 1), dx=(1 / 64, 1, 1),
                                bc_lo=(1, 0, 0), bc_hi=(1, 0, 0))
    assert with_walls > fld.fld_workspace_bytes(p0) > 0
    bad = [
        dict(good, bc_value_hi=(0.0, 0, 0)),
        dict(good, bc_value_hi=(float("nan"), 0, 0)),
        dict(good, bc_lo=(0, 0, 0)),  # periodic on the other side
        dict(good, precision=fld.FLD_PREC_FP32_IR),
        dict(good, krylov=1),
        dict(good, bc_lo=(3, 0, 0)),
    ]
    for kw in bad:
        p = fld.fld_params_default(**kw)
        assert fld.fld_workspace_bytes(p) == 0, kw
        st = lib.fld_setup(ctypes.byref(p), ctypes.c_void_p(256), 1 << 30,
                           None, ctypes.byref(out))
        assert st == fld.FLD_ERR_INVALID_ARG, kw
    p = make_params(2, (16, 16), (0.1, 0.1), ("periodic", "neumann"),
                    dirichlet={(1, 0): 3.0, (1, 1): 1.5})
    assert list(p.bc_lo)[:2] == [0, D] and list(p.bc_hi)[:2] == [0, D]
    assert p.bc_value_lo[1] == 3.0 and p.bc_value_hi[1] == 1.5
    assert fld.fld_workspace_bytes(p) > 0


def test_held_cells_validation():
    """Held cells (fld_set_held): held_cells 0 or 1, an FP64 V-cycle solve,
    not batched; the workspace grows by the coarse levels' masks."""
    lib = fld.load()
    out = ctypes.c_void_p()
    good = dict(ndim=2, n=(32, 32, 1), dx=(1 / 32, 1 / 32, 1),
                bc_lo=(0, 1, 0), bc_hi=(0, 1, 0), held_cells=1)
    p = fld.fld_params_default(**good)
    p0 = fld.fld_params_default(**dict(good, held_cells=0))
    assert fld.fld_workspace_bytes(p) > fld.fld_workspace_bytes(p0) > 0
    for kw in [dict(good, held_cells=2), dict(good, krylov=1),
               dict(good, precision=fld.FLD_PREC_FP32_IR),
               dict(good, guess=fld.FLD_GUESS_LEARNED)]:
        p = fld.fld_params_default(**kw)
        assert fld.fld_workspace_bytes(p) == 0, kw
        st = lib.fld_setup(ctypes.byref(p), ctypes.c_void_p(256), 1 << 30,
                           None, ctypes.byref(out))
        assert st == fld.FLD_ERR_INVALID_ARG, kw
    # no context: fld_step_noalloc and the batch take no held cells
    p = fld.fld_params_default(**good)
    st = lib.fld_step_noalloc(ctypes.byref(p), ctypes.c_double(0.1), None,
                              None, None, None, None, None)
    assert st == fld.FLD_ERR_INVALID_ARG
    assert "held" in lib.fld_last_error(None).decode()
    assert fld.fld_workspace_bytes_batch([p, p]) == 0
    assert lib.fld_set_held(None, None, None) == fld.FLD_ERR_INVALID_ARG


def test_amr_validation():
    """Block-adaptive set-up: a 2D FP64 grid whose sides are multiples of
    the block, distinct refined blocks inside it."""
    good = fld.fld_params_default(ndim=2, n=(32, 16, 1), dx=(1 / 32, 1 / 32, 1),
                                  bc_lo=(0, 1, 0), bc_hi=(0, 1, 0))
    assert fld.fld_amr_workspace_bytes(good, 8, [(1, 1), (2, 0)]) > \
        fld.fld_amr_workspace_bytes(good, 8, []) > 0
    assert fld.fld_amr_workspace_bytes(good, 8, [(4, 0)]) == 0   # outside
    assert fld.fld_amr_workspace_bytes(good, 8, [(1, 1), (1, 1)]) == 0
    assert fld.fld_amr_workspace_bytes(good, 5, []) == 0         # 32 % 5
    assert fld.fld_amr_workspace_bytes(good, 1, []) == 0
    for kw in [dict(ndim=3, n=(32, 16, 8)), dict(precision=1), dict(krylov=1),
               dict(guess=fld.FLD_GUESS_LEARNED), dict(held_cells=1),
               dict(bc_hi=(0, 2, 0), bc_value_hi=(0, 1.0, 0))]:
        base = dict(ndim=2, n=(32, 16, 1), dx=(1 / 32, 1 / 32, 1),
                    bc_lo=(0, 1, 0), bc_hi=(0, 1, 0))
        base.update(kw)
        p = fld.fld_params_default(**base)
        assert fld.fld_amr_workspace_bytes(p, 8, []) == 0, kw
    with pytest.raises(fld.FldError):
        fld.fld_amr_setup(fld.fld_params_default(ndim=1, n=(32, 1, 1)), 8, [])


def test_status_strings():
    assert fld.status_str(fld.FLD_OK) == "FLD_OK"
    assert fld.status_str(fld.FLD_ERR_NOT_CONVERGED) == "FLD_ERR_NOT_CONVERGED"
