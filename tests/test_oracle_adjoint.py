"""Pins for the oracle's adjoint gradients: central finite differences of the loss."""

import numpy as np

from oracle import adjoint, fdweights as fw, transfer
from workloads import disk_mesh, fourier_rhs, grid_for_box


def _setup():
    mesh = disk_mesh(seed=9, n_boundary=24, spacing=0.22)
    g = grid_for_box(2, 24, R=1.1)
    s = 0.6
    T = fw.filon_richardson(s, 2, 2 * g.N, 256)
    f = fourier_rhs(31, g)
    tr = transfer.Transfer(mesh.X, mesh.elems, 2, g.N, g.R, g.center)
    rng = np.random.default_rng(2)
    ut = rng.standard_normal(tr.J.size) * 0.1
    return mesh, g, s, T, f, tr, ut


def _loss(tr, T, s, f, ut):
    uJ, _ = adjoint.forward_dense(tr, T, s, f)
    return 0.5 * np.sum((uJ - ut) ** 2), uJ


def test_grad_f_matches_central_differences():
    mesh, g, s, T, f, tr, ut = _setup()
    L0, uJ = _loss(tr, T, s, f, ut)
    gf, _ = adjoint.gradients(tr, T, s, f, uJ, uJ - ut)
    rng = np.random.default_rng(4)
    inside = tr.inside
    for k in rng.choice(inside, 6, replace=False):
        e = np.zeros(f.size)
        e[k] = 1.0
        step = 1e-3
        lp, _ = _loss(tr, T, s, f + step * e.reshape(f.shape), ut)
        lm, _ = _loss(tr, T, s, f - step * e.reshape(f.shape), ut)
        fd = (lp - lm) / (2 * step)              # exact up to rounding: L is quadratic in f
        assert abs(fd - gf.ravel()[k]) <= 1e-8 * max(1e-12, abs(fd)) + 1e-15
    outside = np.nonzero(tr.elem < 0)[0]
    assert np.all(gf.ravel()[outside] == 0)


def test_grad_X_matches_central_differences():
    mesh, g, s, T, f, tr, ut = _setup()
    L0, uJ = _loss(tr, T, s, f, ut)
    _, gX = adjoint.gradients(tr, T, s, f, uJ, uJ - ut)
    step = 1e-6
    checked = 0
    for j in list(tr.J[:6]) + [int(np.nonzero(tr.bnd)[0][0])]:
        for a in range(2):
            vals = []
            for sg in (+1, -1):
                X2 = mesh.X.copy()
                X2[j, a] += sg * step
                tr2 = transfer.Transfer(X2, mesh.elems, 2, g.N, g.R, g.center, elem_of_node=tr.elem)
                vals.append(_loss(tr2, T, s, f, ut)[0])
            fd = (vals[0] - vals[1]) / (2 * step)
            assert abs(fd - gX[j, a]) <= 1e-5 * max(abs(fd), 1e-8) + 1e-9, (j, a, fd, gX[j, a])
            checked += 1
    assert checked == 14
