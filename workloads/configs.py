"""The five named workloads, as concrete seeded inputs.

Each entry returns plain numpy arrays (mesh, grid, orders s, right-hand
sides); nothing here computes any part of the method.

  c1  2D unit disk, ~1k vertices, 64x64 grid on [-1,1]^2, s = 0.5, f = 1
  c2  2D L-shape [-1,1]^2 minus [0,1]^2, ~65k vertices graded toward the
      corner, 1024x1024 grid, s in {0.25, 0.75}, 16-mode Fourier f
  c3  3D unit ball, ~200k vertices, 256^3 grid, s = 0.5, f = 1
  c4  64 star-shaped polygons (2k..100k vertices, log-uniform), grids
      128^2..1024^2, s ~ U[0.1, 0.9], 16 Fourier right-hand sides each
  c5  one star-shaped polygon, 250k vertices, 2048^2 grid, s = 0.6
"""

from __future__ import annotations

import functools
import math

import numpy as np

from .grids import grid_for_box
from .meshes import ball_mesh, disk_mesh, lshape_mesh, star_mesh, star_radius_fn
from .rhs import constant_rhs, fourier_rhs


@functools.lru_cache(maxsize=8)
def _c1():
    mesh = disk_mesh(seed=1001)
    grid = grid_for_box(2, 64, R=1.0)
    return dict(name="c1-disk", mesh=mesh, grid=grid, s=[0.5], f=[constant_rhs(grid)], tol=1e-10,
                precond="IC1_9")


@functools.lru_cache(maxsize=2)
def _c2():
    mesh = lshape_mesh(seed=1002)
    grid = grid_for_box(2, 1024, R=1.0)
    f = fourier_rhs(1002, grid, box_lo=[-1.0, -1.0], box_len=[2.0, 2.0])
    return dict(name="c2-lshape", mesh=mesh, grid=grid, s=[0.25, 0.75], f=[f], tol=1e-8,
                precond="IC1_9")


@functools.lru_cache(maxsize=1)
def _c3():
    mesh = ball_mesh(seed=1003)
    grid = grid_for_box(3, 256, R=1.0)
    return dict(name="c3-ball", mesh=mesh, grid=grid, s=[0.5], f=[constant_rhs(grid)], tol=1e-8,
                precond="IC1_27")


def _c4_member(i, seed=1004):
    ss = np.random.SeedSequence(seed).spawn(64)[i]
    rng = np.random.default_rng(ss)
    nv = int(round(math.exp(rng.uniform(math.log(2000), math.log(100000)))))
    s = float(rng.uniform(0.1, 0.9))
    mseed = int(rng.integers(1 << 30))
    n = int(np.clip(2 ** round(math.log2(math.sqrt(8 * nv))), 128, 1024))
    rfun = star_radius_fn(mseed)
    rmax = float(rfun(np.linspace(0, 2 * np.pi, 4096, endpoint=False)).max())
    R = 1.1 * rmax
    grid = grid_for_box(2, n, R=R)
    rhs_seeds = [int(x) for x in rng.integers(1 << 30, size=16)]
    return dict(nv=nv, s=s, mesh_seed=mseed, grid=grid, rhs_seeds=rhs_seeds)


def c4_plan(seed=1004, count=64):
    return [_c4_member(i, seed) for i in range(count)]


def c4_problem(member):
    mesh = star_mesh(member["mesh_seed"], member["nv"])
    grid = member["grid"]
    fs = [fourier_rhs(sd, grid, box_lo=[-grid.R, -grid.R], box_len=[2 * grid.R] * 2)
          for sd in member["rhs_seeds"]]
    return dict(mesh=mesh, grid=grid, s=member["s"], f=fs)


@functools.lru_cache(maxsize=1)
def _c5():
    rfun = star_radius_fn(1005)
    rmax = float(rfun(np.linspace(0, 2 * np.pi, 4096, endpoint=False)).max())
    mesh = star_mesh(1005, 250000)
    grid = grid_for_box(2, 2048, R=1.1 * rmax)
    f = fourier_rhs(1005 + 1, grid)
    return dict(name="c5-star", mesh=mesh, grid=grid, s=[0.6], f=[f], tol=1e-8, precond="IC1_9")


def config_inputs(name: str):
    return {"c1": _c1, "c2": _c2, "c3": _c3, "c5": _c5}[name]()
