"""CPU checks of the C ABI library: it loads, exports every declared symbol, and its
host-side pieces (Gaunt table, LIZ construction, argument checking) match the oracle."""

import ctypes
import os
import re

import numpy as np
import pytest

import synthetic
from oracle import liz as oliz
from oracle import special

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(lsms_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    from paper_2311_12134_amd import _lib
    L = ctypes.CDLL(_lib.LIB_PATH)
    names = _declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib._PROTOS), "ctypes prototypes and header disagree"


def test_gaunt_table_matches_oracle():
    import paper_2311_12134_amd as P
    G = P.gaunt_table()
    C = special.gaunt_table(3, 3, 6)
    assert np.abs(G - C).max() < 1e-14
    assert (np.abs(G) > 0).sum() == 708


@pytest.mark.parametrize("name", ["fcc32", "bcc16", "bcc250", "bcc1940"])
def test_liz_matches_oracle_exactly(name):
    import paper_2311_12134_amd as P
    w = synthetic.workload(name)
    L = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    o = oliz.build_liz(w["pos"], w["cell"], w["r_liz"])
    assert np.array_equal(L.ptr, o[0])
    assert np.array_equal(L.atom, o[1])
    assert np.array_equal(L.pos, o[2])  # bitwise: same IEEE operations in the same order


def test_liz_fcc4000_sizes():
    import paper_2311_12134_amd as P
    w = synthetic.workload("fcc4000")
    L = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    assert (np.diff(L.ptr) == 135).all()


def _same_lists(L, o, centres):
    for i in centres:
        a, b, c, d = int(L.ptr[i]), int(L.ptr[i + 1]), int(o[0][i]), int(o[0][i + 1])
        assert b - a == d - c
        assert np.array_equal(L.atom[a:b], o[1][c:d]) and np.array_equal(L.pos[a:b], o[2][c:d]), i


@pytest.mark.parametrize("name,full", [("fcc4000", True), ("fcc4000", False), ("bcc16000", False)])
def test_liz_matches_oracle_on_sampled_centres(name, full):
    """The large workloads' LIZ (full build and the centre-subset build) against the oracle's
    own construction for seeded centres, bitwise."""
    import paper_2311_12134_amd as P
    w = synthetic.workload(name)
    n = len(w["pos"])
    centres = sorted(set([0, n - 1, n // 2 + 7] + list(np.random.default_rng(5).choice(n, 12, replace=False))))
    L = P.build_liz(w["pos"], w["cell"], w["r_liz"], centres=None if full else centres)
    o = oliz.build_liz(w["pos"], w["cell"], w["r_liz"], centres=centres)
    _same_lists(L, o, centres)
    assert all(int(o[0][i + 1] - o[0][i]) == 0 for i in range(n) if i not in set(centres))


@pytest.mark.parametrize("pos,r", [
    (np.array([[0, 0, 0], [3.0, 0, 0], [0, 4.0, 0], [10.0, 0, 0]]), 5.5),
    (np.array([[0.0, 0.0, 0.0], [4.2, 0.3, 0.1], [0.4, 4.1, -0.3], [40.0, 0.0, 0.0], [47.0, 1.0, 0.0]]), 7.5),
    (np.array([[0.0, 0.0, 0.0], [4.2, 0.3, 0.1], [0.4, 4.1, -0.3], [40.0, 0.0, 0.0], [47.0, 1.0, 0.0]]), 5.0)])
def test_liz_open_cluster(pos, r):
    import paper_2311_12134_amd as P
    L = P.build_liz(pos, None, r)
    o = oliz.build_liz(pos, None, r)
    assert np.array_equal(L.ptr, o[0]) and np.array_equal(L.atom, o[1]) and np.array_equal(L.pos, o[2])


def test_liz_argument_errors():
    import paper_2311_12134_amd as P
    from paper_2311_12134_amd._lib import LsmsError
    with pytest.raises(LsmsError) as e:
        P.build_liz(np.zeros((2, 3)), None, 1.0)
    assert e.value.code == -1 and "coincident" in str(e.value)
    with pytest.raises(LsmsError):
        P.build_liz(np.zeros((1, 3)), None, -1.0)
    with pytest.raises(LsmsError):
        P.build_liz(np.array([[np.nan, 0, 0]]), None, 1.0)
    pos, cell = synthetic.fcc_supercell(7.0, 4)
    with pytest.raises(LsmsError):
        P.build_liz(pos, cell, 4.0 * 7.0)  # > 256 members


def test_liz_capacity_reporting():
    from paper_2311_12134_amd._lib import lib
    pos, cell = synthetic.fcc_supercell(7.7, 2)
    ptr = np.zeros(33, dtype=np.int64)
    needed = ctypes.c_int64(0)
    atom = np.zeros(10, dtype=np.int32)
    disp = np.zeros((10, 3))
    rc = lib().lsms_build_liz(None, 32, pos.ctypes.data_as(ctypes.c_void_p), cell.ctypes.data_as(ctypes.c_void_p),
                              1.1 * 7.7, 10, ptr.ctypes.data_as(ctypes.c_void_p), atom.ctypes.data_as(ctypes.c_void_p),
                              disp.ctypes.data_as(ctypes.c_void_p), ctypes.byref(needed))
    assert rc == -2 and needed.value == 32 * 19


def test_create_rejects_lmax_before_touching_a_device():
    from paper_2311_12134_amd._lib import lib
    h = ctypes.c_void_p()
    assert lib().lsms_create(0, 4, 0, ctypes.byref(h)) == -1
    assert b"lmax" in lib().lsms_last_error()


def test_liz_subset_matches_full_build():
    import paper_2311_12134_amd as P
    w = synthetic.workload("bcc250")
    full = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    cen = [3, 100, 100, 249]
    sub = P.build_liz(w["pos"], w["cell"], w["r_liz"], centres=cen)
    sizes = np.diff(sub.ptr)
    assert (sizes[[3, 100, 249]] > 0).all() and sizes.sum() == sum(np.diff(full.ptr)[[3, 100, 249]])
    for i in range(250):
        if i in cen:
            a, b = slice(full.ptr[i], full.ptr[i + 1]), slice(sub.ptr[i], sub.ptr[i + 1])
            assert np.array_equal(full.atom[a], sub.atom[b]) and np.array_equal(full.pos[a], sub.pos[b])
        else:
            assert sizes[i] == 0


def test_liz_paper_scale_membership():
    """bcc16000 at r_LIZ = 4.9a: 965 members, exactly the images within the radius
    (brute force over periodic images for one centre)."""
    import paper_2311_12134_amd as P
    w = synthetic.workload("bcc16000")
    L = P.build_liz(w["pos"], w["cell"], w["r_liz"], centres=[7])
    assert np.diff(L.ptr)[7] == 965
    d = w["pos"][None, :, :] - w["pos"][7][None, None, :]
    shifts = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)], dtype=float)
    imgs = (d + (shifts @ w["cell"])[:, None, :]).reshape(-1, 3)
    r = np.linalg.norm(imgs, axis=1)
    assert int((r < w["r_liz"]).sum()) == 965
    got = np.sort(np.linalg.norm(L.pos[L.ptr[7]:L.ptr[8]], axis=1))
    assert np.allclose(got, np.sort(r[r < w["r_liz"]]), rtol=0, atol=1e-9)


def test_liz_above_limit_is_rejected():
    """r_LIZ = 5.0a in bcc gives 1037 sites, more than the 1024 the solves accept."""
    import paper_2311_12134_amd as P
    from paper_2311_12134_amd._lib import LsmsError
    w = synthetic.workload("bcc16000")
    with pytest.raises(LsmsError):
        P.build_liz(w["pos"], w["cell"], 5.0 * w["a"], centres=[0])


def test_header_is_plain_c_and_links(tmp_path):
    """include/lsms_kkr.h compiles as C99 and a C program linked against the library can
    call the host entry points (LIZ construction, Gaunt table, error text)."""
    import shutil
    import subprocess
    from paper_2311_12134_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "abi_check.c"
    src.write_text(r"""
#include <stdio.h>
#include "lsms_kkr.h"
int main(void) {
  double pos[6] = {0, 0, 0, 3.0, 0, 0};
  int64_t ptr[3], needed = 0;
  int32_t atom[4];
  double disp[12];
  double gaunt[16 * 16 * 49];
  int rc = lsms_build_liz(NULL, 2, pos, NULL, 4.0, 4, ptr, atom, disp, &needed);
  if (rc != LSMS_OK || needed != 4 || ptr[1] != 2 || ptr[2] != 4 || atom[0] != 0 || atom[1] != 1) return 1;
  if (lsms_build_liz(NULL, 2, pos, NULL, -1.0, 4, ptr, atom, disp, &needed) != LSMS_E_ARG) return 2;
  if (lsms_last_error()[0] == 0) return 3;
  if (lsms_gaunt_table(gaunt) != LSMS_OK || gaunt[0] < 0.28 || gaunt[0] > 0.29) return 4;
  printf("ok %lld\n", (long long)needed);
  return 0;
}
""")
    exe = tmp_path / "abi_check"
    libdir = os.path.dirname(_lib.LIB_PATH)
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                    "-L", libdir, "-llsms_kkr", "-Wl,-rpath," + libdir], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "ok 4", (out.returncode, out.stdout, out.stderr)
