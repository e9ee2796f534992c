"""Host-side checks of the C ABI (no GPU needed): libslnk.so loads, exports every function that
include/slnk.h declares, the ctypes binding mirrors the header's structs field by field, and
argument validation rejects bad parameters before any device work."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slnk.h")
HEADER3 = os.path.join(ROOT, "include", "slnk3.h")


@pytest.fixture(scope="module")
def pkg():
    import paper_1604_02153_amd as p
    if not os.path.exists(p.library_path()):
        from paper_1604_02153_amd import build
        build.build()
    p.load_library()
    return p


def declared_functions(header=HEADER, prefix="slnk_"):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(" + prefix + r"\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("slnk_create", "slnk_gradient", "slnk_hessian_matvec", "slnk_precond_apply",
                     "slnk_newton_solve", "slnk_objective", "slnk_split_matvec"):
        assert required in names


def test_library_exports_every_declared_symbol(pkg):
    lib = ctypes.CDLL(pkg.library_path())
    names = declared_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing
    assert sorted(pkg.EXPORTS) == names  # the binding covers exactly the header
    names3 = declared_functions(HEADER3, "slnk3_")
    assert "slnk3_newton_solve" in names3 and "slnk3_hessian_matvec" in names3
    assert not [n for n in names3 if not hasattr(lib, n)]
    assert sorted(pkg.EXPORTS3) == names3


LAYOUT_PROGRAM = r"""
#include <stddef.h>
#include <stdio.h>
#include "slnk3.h"
#define F(T, m) printf(#T " " #m " %zu %zu\n", offsetof(T, m), sizeof(((T*)0)->m))
int main(void) {
  printf("slnk_params size %zu 0\n", sizeof(slnk_params));
  F(slnk_params, n1); F(slnk_params, n2); F(slnk_params, nt); F(slnk_params, reg); F(slnk_params, beta);
  F(slnk_params, prec); F(slnk_params, pc); F(slnk_params, cheb_iters); F(slnk_params, lanczos_steps);
  F(slnk_params, emax_safety); F(slnk_params, lanczos_seed); F(slnk_params, use_graphs); F(slnk_params, batch);
  F(slnk_params, sl_path); F(slnk_params, hessian); F(slnk_params, proj);
  F(slnk_params, coarse_solver); F(slnk_params, coarse_eps); F(slnk_params, transport);
  printf("slnk_solve_opts size %zu 0\n", sizeof(slnk_solve_opts));
  F(slnk_solve_opts, max_newton); F(slnk_solve_opts, gtol_rel); F(slnk_solve_opts, gtol_abs);
  F(slnk_solve_opts, max_pcg); F(slnk_solve_opts, armijo_c1); F(slnk_solve_opts, max_halvings);
  printf("slnk_solve_report size %zu 0\n", sizeof(slnk_solve_report));
  F(slnk_solve_report, status); F(slnk_solve_report, newton_iters); F(slnk_solve_report, pcg_iters);
  F(slnk_solve_report, matvecs); F(slnk_solve_report, coarse_matvecs); F(slnk_solve_report, line_search_evals);
  F(slnk_solve_report, g0_inf); F(slnk_solve_report, g0_two); F(slnk_solve_report, emin);
  F(slnk_solve_report, emax); F(slnk_solve_report, grel); F(slnk_solve_report, J); F(slnk_solve_report, pcg);
  F(slnk_solve_report, time_total_ms); F(slnk_solve_report, time_gradient_ms); F(slnk_solve_report, time_pcg_ms);
  F(slnk_solve_report, time_precond_ms); F(slnk_solve_report, time_linesearch_ms);
  F(slnk_solve_report, time_to_stop_ms); F(slnk_solve_report, fallback); F(slnk_solve_report, cheb_reestimates);
  printf("slnk_unet_params size %zu 0\n", sizeof(slnk_unet_params));
  F(slnk_unet_params, height); F(slnk_unet_params, width); F(slnk_unet_params, levels);
  F(slnk_unet_params, base_channels); F(slnk_unet_params, max_batch); F(slnk_unet_params, seed);
  F(slnk_unet_params, start_kmax);
  printf("slnk3_params size %zu 0\n", sizeof(slnk3_params));
  F(slnk3_params, n1); F(slnk3_params, n2); F(slnk3_params, n3); F(slnk3_params, nt); F(slnk3_params, reg);
  F(slnk3_params, beta); F(slnk3_params, prec); F(slnk3_params, proj); F(slnk3_params, sl_path);
  F(slnk3_params, pc); F(slnk3_params, cheb_iters); F(slnk3_params, lanczos_steps); F(slnk3_params, emax_safety);
  F(slnk3_params, lanczos_seed); F(slnk3_params, hessian); F(slnk3_params, coarse_solver);
  F(slnk3_params, coarse_eps); F(slnk3_params, transport);
  return 0;
}
"""


def test_ctypes_structs_match_the_header(pkg, tmp_path):
    src = tmp_path / "layout.c"
    exe = tmp_path / "layout"
    src.write_text(LAYOUT_PROGRAM)
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    structs = {"slnk_params": pkg.Params, "slnk_solve_opts": pkg.SolveOpts, "slnk_solve_report": pkg.SolveReport,
               "slnk_unet_params": pkg.UNetParams, "slnk3_params": pkg.Params3}
    seen = {k: [] for k in structs}
    for line in filter(None, out):
        name, field, off, size = line.split()
        cls = structs[name]
        if field == "size":
            assert ctypes.sizeof(cls) == int(off), name
            continue
        desc = getattr(cls, field)
        assert (desc.offset, desc.size) == (int(off), int(size)), (name, field)
        seen[name].append(field)
    for name, cls in structs.items():
        assert [f[0] for f in cls._fields_] == seen[name]


def test_defaults_are_the_paper_settings(pkg):
    lib = pkg.load_library()
    p = pkg.Params()
    lib.slnk_default_params(ctypes.byref(p))
    assert (p.cheb_iters, p.lanczos_steps, p.batch, p.reg, p.pc) == (10, 30, 1, 2, 2)
    o = pkg.SolveOpts()
    lib.slnk_default_opts(ctypes.byref(o))
    assert (o.gtol_rel, o.gtol_abs) == (1e-2, 1e-5)


@pytest.mark.parametrize("change", [dict(n1=30, n2=34), dict(nt=0), dict(batch=0), dict(reg=4), dict(beta=0.0),
                                    dict(prec=7), dict(pc=3), dict(n1=2048 * 2), dict(n1=2048), dict(cheb_iters=0),
                                    dict(sl_path=4), dict(lanczos_steps=1001)])
def test_create_rejects_bad_parameters_before_device_work(pkg, change):
    lib = pkg.load_library()
    p = pkg.Params()
    lib.slnk_default_params(ctypes.byref(p))
    for k, v in change.items():
        setattr(p, k, v)
    ctx = ctypes.c_void_p()
    assert lib.slnk_create(ctypes.byref(p), None, ctypes.byref(ctx)) == 1  # SLNK_EINVAL
    assert not ctx.value


def test_calls_reject_null_arguments(pkg):
    lib = pkg.load_library()
    assert lib.slnk_create(None, None, None) == 1
    assert lib.slnk_gradient(None, None, None, None) == 1
    assert lib.slnk_newton_solve(None, None, None, None) == 1
    assert lib.slnk_workspace_bytes(None) == 0
    assert lib.slnk_last_error(None) == b"null context"


@pytest.mark.parametrize("change", [dict(levels=1), dict(base_channels=16), dict(height=100), dict(max_batch=0),
                                    dict(height=32, width=32, levels=4)])
def test_unet_create_rejects_bad_shapes(pkg, change):
    lib = pkg.load_library()
    p = pkg.UNetParams()
    lib.slnk_unet_default_params(ctypes.byref(p))
    assert (p.height, p.levels, p.base_channels) == (256, 4, 32)
    for k, v in change.items():
        setattr(p, k, v)
    u = ctypes.c_void_p()
    assert lib.slnk_unet_create(ctypes.byref(p), None, ctypes.byref(u)) == 1
    assert not u.value


@pytest.mark.parametrize("change", [dict(n1=24), dict(n3=1024), dict(n2=4), dict(nt=0), dict(reg=0), dict(beta=-1.0),
                                    dict(prec=2), dict(proj=2), dict(sl_path=2), dict(pc=3),
                                    dict(pc=2, n1=8), dict(pc=2, cheb_iters=0), dict(pc=2, emax_safety=0.5),
                                    dict(pc=2, lanczos_steps=1001), dict(hessian=2),
                                    dict(coarse_solver=2), dict(pc=2, coarse_solver=1, coarse_eps=0.0),
                                    dict(pc=2, coarse_solver=1, coarse_eps=1.0), dict(transport=2),
                                    dict(pc=2, transport=1)])
def test_create3_rejects_bad_parameters_before_device_work(pkg, change):
    lib = pkg.load_library()
    p = pkg.Params3()
    lib.slnk3_default_params(ctypes.byref(p))
    assert (p.n1, p.n2, p.n3, p.nt, p.reg, p.hessian, p.coarse_solver, p.coarse_eps, p.transport) == \
        (64, 64, 64, 4, 2, 0, 0, 0.1, 0)
    for k, v in change.items():
        setattr(p, k, v)
    ctx = ctypes.c_void_p()
    assert lib.slnk3_create(ctypes.byref(p), None, ctypes.byref(ctx)) == 1  # SLNK_EINVAL
    assert not ctx.value
    assert lib.slnk3_gradient(None, None, None, None) == 1
    assert lib.slnk3_workspace_bytes(None) == 0
    assert lib.slnk3_last_error(None) == b"null context"
