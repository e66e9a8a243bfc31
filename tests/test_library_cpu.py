"""CPU checks of the C ABI library: it is built, loads, exports every entry
point include/sdg.h declares, and its structs have the layout the binding
assumes (checked against the C compiler).  No device calls."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sdg.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sdg_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def sdg():
    from paper_1607_03777_amd import sdg as s
    if not os.path.exists(s.LIBPATH):
        from paper_1607_03777_amd import build
        build.build()
    s.lib()
    return s


def test_exports_every_declared_symbol(sdg):
    names = declared()
    assert len(names) >= 25
    out = subprocess.run(["nm", "-D", "--defined-only", sdg.LIBPATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert set(sdg.PROTOTYPES) == set(names)


def test_struct_layout_matches_c(sdg, tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "sdg.h"
int main(void) {
  printf("%zu %zu %zu\\n", sizeof(sdg_mesh), sizeof(sdg_options), sizeof(sdg_stats));
  printf("%zu %zu %zu %zu\\n", offsetof(sdg_mesh, lx), offsetof(sdg_mesh, k), offsetof(sdg_mesh, bc),
         offsetof(sdg_options, cheb_lo));
  printf("%zu %zu %zu\\n", offsetof(sdg_options, prec_smoother), offsetof(sdg_options, seed),
         offsetof(sdg_stats, rel_residual));
  printf("%zu %zu %zu %zu\\n", sizeof(sdg_server_config), offsetof(sdg_server_config, mem_budget),
         sizeof(sdg_req_info), offsetof(sdg_req_info, bytes));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    py = [ctypes.sizeof(sdg.sdg_mesh), ctypes.sizeof(sdg.sdg_options), ctypes.sizeof(sdg.sdg_stats),
          sdg.sdg_mesh.lx.offset, sdg.sdg_mesh.k.offset, sdg.sdg_mesh.bc.offset,
          sdg.sdg_options.cheb_lo.offset, sdg.sdg_options.prec_smoother.offset,
          sdg.sdg_options.seed.offset, sdg.sdg_stats.rel_residual.offset,
          ctypes.sizeof(sdg.sdg_server_config), sdg.sdg_server_config.mem_budget.offset,
          ctypes.sizeof(sdg.sdg_req_info), sdg.sdg_req_info.bytes.offset]
    assert vals == py


def test_default_options_are_paper_values(sdg):
    import json
    p = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_parameters.json")))
    o = sdg.make_options()
    assert o.cheb_lo == p["chebyshev_lo"]["value"] and o.cheb_hi == p["chebyshev_hi"]["value"]
    assert o.eig_steps == p["eig_gmres_steps"]["value"]
    assert o.smooth_dg == p["smooth_p_level"]["value"] and o.smooth_h == p["smooth_h_level"]["value"]
    assert o.inner_rtol == p["rtol_inner"]["value"]


def test_required_bytes_is_host_only_and_monotone(sdg):
    o = sdg.make_options()
    small = sdg.sdg_required_bytes(sdg.make_mesh(16, 16, 2), o, 0)
    big = sdg.sdg_required_bytes(sdg.make_mesh(64, 64, 4), o, 0)
    stokes = sdg.sdg_required_bytes(sdg.make_mesh(64, 64, 4), o, 1)
    assert 0 < small < big < stokes
    assert sdg.sdg_required_bytes(sdg.make_mesh(0, 4, 2), o, 0) == 0
    assert sdg.sdg_required_bytes(sdg.make_mesh(4, 4, 9), o, 0) == 0


@pytest.mark.parametrize("prec_s,width", [(0, 0), (1, 4), (2, 2)])
def test_required_bytes_bounds_the_element_blocks(sdg, prec_s, width):
    """The admission figure is an upper bound: every element block counted as
    distinct (a viscosity that varies per element leaves nothing to
    deduplicate), each stored as its FP64 inverse and, in low precision, as
    the packed FP64 factor plus the factor in the storage type as a lower
    triangle of 2 x 2 quads, NB (NB + 2) / 2 values (the setup's
    allocations)."""
    n, k, nbatch = 64, 5, 3
    NB = 2 * (k + 1) ** 2
    o = sdg.make_options(prec_apply=1 if prec_s else 0, prec_smoother=prec_s)
    need = sdg.sdg_required_bytes_batch(sdg.make_mesh(n, n, k), o, 0, nbatch)
    nblk = n * n * nbatch
    blocks = nblk * NB * NB * 8
    if prec_s:
        blocks += nblk * (NB * (NB + 1) // 2 * 8 + NB * (NB + 2) // 2 * width)
    vectors = nbatch * n * n * NB * 8 * 7  # at least the CG and cycle vectors
    assert need >= blocks + vectors
