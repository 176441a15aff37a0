"""Argument checks of mln_pstd_init (CPU: every case returns before any
device call)."""
import ctypes
import math

import numpy as np
import pytest

from paper_1710_09799_amd import mln
from paper_1710_09799_amd import workloads as W


def _init(media, grid):
    L = mln.load()
    meds = (mln._Medium * len(media))()
    keep = []
    for i, m in enumerate(media):
        ma = mln._MediumArgs(m)
        keep.append(ma)
        meds[i] = ma.s
    g = mln._Grid(grid.nx, grid.nt, grid.dx, grid.dt, grid.med_begin, grid.med_end, grid.eps_r, grid.mu_r,
                  grid.sigma)
    h = ctypes.c_void_p()
    rc = L.mln_pstd_init(len(media), meds, ctypes.byref(g), None, None, None, None, ctypes.byref(h))
    assert not h.value
    return rc, L.mln_last_error().decode()


def _grid(nx=256, dt=None, mb=64, me=192):
    return W.Grid(nx=nx, nt=10, dx=W.DX_PSTD, dt=W.DT_PSTD if dt is None else dt, med_begin=mb, med_end=me)


def test_rejects_grids_that_are_not_powers_of_two():
    rc, msg = _init([W.random_medium(2, 1)], _grid(nx=200))
    assert rc == -1 and "power of two" in msg
    rc, _ = _init([W.random_medium(2, 1)], _grid(nx=32, mb=4, me=20))
    assert rc == -1


@pytest.mark.parametrize("n,nx", [(2, 8192), (3, 8192), (4, 4096), (6, 2048)])
def test_rejects_grids_beyond_the_built_size(n, nx):
    rc, msg = _init([W.random_medium(n, 1)], _grid(nx=nx, mb=10, me=20))
    assert rc == -8 and "too large" in msg


def test_rejects_unbuilt_level_count_and_mixed_media():
    rc, _ = _init([W.random_medium(5, 1)], _grid())
    assert rc == -8
    rc, msg = _init([W.random_medium(2, 1), W.random_medium(3, 1)], _grid())
    assert rc == -1 and "level count" in msg


def test_leapfrog_stability_limit():
    """c dt kappa_max / 2 < 1 with kappa_max = 2 pi (nx/2 - 1) / (nx dx):
    just above the limit is rejected (MLN_ECOURANT)."""
    nx = 256
    kmax = 2 * math.pi * (nx // 2 - 1) / (nx * W.DX_PSTD)
    c0 = 1.0 / math.sqrt(8.8541878128e-12 * 1.25663706212e-6)
    dt_lim = 2.0 / (c0 * kmax)
    rc, _ = _init([W.random_medium(2, 1)], _grid(nx=nx, dt=dt_lim * 1.001))
    assert rc == -4


def test_rejects_medium_outside_the_grid():
    rc, _ = _init([W.random_medium(2, 1)], _grid(mb=0, me=10))
    assert rc == -1
    rc, _ = _init([W.random_medium(2, 1)], _grid(mb=10, me=256))
    assert rc == -1
