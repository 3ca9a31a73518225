"""Pins of the oracle's hand-written reverse mode against its own forward
step through central finite differences (the transpose identity
<lam, J d> = <J^T lam, d>), for each kind of boundary, plus the objective
gradient and the equilibrium-initialisation VJP. The paper has no adjoint;
these checks tie the reverse sweep to the forward step it differentiates."""
import numpy as np
import pytest

from paper_1010_4124_amd import inputs

P, F, R = 0, 1, 2


def _near_eq_f(orc, p, seed):
    r, ux, uy, T = inputs.random_fields(p.nx, p.ny, seed, smooth=False)
    f = orc.init(p, r, ux, uy, T)
    return f * (1.0 + 0.05 * inputs.random_like(f.shape, seed + 100))


def _fd(fun, x, d, h=1e-6):
    """Central difference with one Richardson extrapolation (error O(h^4))."""
    d1 = (fun(x + h * d) - fun(x - h * d)) / (2 * h)
    d2 = (fun(x + 0.5 * h * d) - fun(x - 0.5 * h * d)) / h
    return (4.0 * d2 - d1) / 3.0


@pytest.mark.parametrize("bc", [(P, P, P, P), (P, P, R, R), (F, F, P, P), (R, R, F, F)])
def test_transpose_identity(orc, bc):
    nx, ny = 11, 9
    side = [(1.1, 0.1, 0.0, 0.9), (0.7, -0.05, 0.02, 1.1), (1.0, 0.0, 0.1, 1.0),
            (0.9, 0.1, -0.1, 0.8)]
    p = orc.OracleParams.make(nx, ny, 2e-2, 2.5e-2, 4e-4, 6e-4, bc, side_state=side)
    f = _near_eq_f(orc, p, 1)
    lam = inputs.random_like(f.shape, 2)
    d = inputs.random_like(f.shape, 3)
    jd = _fd(lambda v: orc.step(p, v), f, d)
    jtl = orc.adjoint_step(p, f, lam, 0.0)
    a, b = np.sum(lam * jd), np.sum(jtl * d)
    assert a == pytest.approx(b, rel=1e-8)
    # and per-component: the full transpose against one-hot directions on a
    # few entries, including ghost-adjacent cells
    for (i, y, x) in [(0, 0, 0), (5, ny - 1, 3), (13, 4, nx - 1), (18, 1, 1), (9, ny - 2, nx - 2)]:
        e = np.zeros_like(f)
        e[i, y, x] = 1.0
        col = _fd(lambda v: orc.step(p, v), f, e)
        assert np.sum(lam * col) == pytest.approx(jtl[i, y, x], rel=1e-6, abs=1e-9)


def test_objective_gradient(orc):
    nx, ny = 10, 8
    p = orc.OracleParams.make(nx, ny, 1e-2, 1e-2, 1e-4, 1e-4, (P, P, R, R))
    f = _near_eq_f(orc, p, 4)
    g = orc.kinetic_y_grad(p, f)
    d = inputs.random_like(f.shape, 5)
    h = 1e-6
    fd = (orc.kinetic_y(p, f + h * d)[0] - orc.kinetic_y(p, f - h * d)[0]) / (2 * h)
    assert np.sum(g * d) == pytest.approx(fd, rel=1e-7)
    # adjoint_step with lam = 0 returns w * dE_y/df
    out = orc.adjoint_step(p, f, np.zeros_like(f), 2.5)
    assert np.allclose(out, 2.5 * g, rtol=1e-14, atol=1e-20)


def test_init_vjp(orc):
    nx, ny = 7, 6
    p = orc.OracleParams.make(nx, ny, 1e-2, 1e-2, 1e-4, 1e-4)
    fields = [np.array(a) for a in inputs.random_fields(nx, ny, 6, smooth=False)]
    lam = inputs.random_like((19, ny, nx), 7)
    g = orc.init_vjp(p, *fields, lam)
    for q in range(4):
        d = inputs.random_like((ny, nx), 8 + q)
        h = 1e-6
        fp = [a.copy() for a in fields]
        fm = [a.copy() for a in fields]
        fp[q] += h * d
        fm[q] -= h * d
        fd = np.sum(lam * (orc.init(p, *fp) - orc.init(p, *fm))) / (2 * h)
        assert np.sum(g[q] * d) == pytest.approx(fd, rel=1e-7)


def test_multistep_reverse_sweep(orc):
    """J(f0) = sum_n w_n E_y(f^n) over 6 steps: the reverse sweep
    lam^n = J_n^T lam^{n+1} + w_n dE_y/df^n gives dJ/df0."""
    nx, ny = 12, 10
    p = orc.OracleParams.make(nx, ny, 1e-2, 1e-2, 2e-4, 2e-4, (P, P, R, R))
    s = inputs.khi(nx, ny, 1e-2, 1e-2, 2e-4, 2e-4, Dv=0.03, Drho=0.03, pert=2e-2)
    f0 = orc.init(p, *s.fields())
    N = 6
    w = np.array([0.0, 0.0, 1.0, 1.0, 0.5, 1.0, 1.0])  # weights on f^0..f^N

    def J(f):
        tot = w[0] * orc.kinetic_y(p, f)[0]
        for n in range(1, N + 1):
            f = orc.step(p, f)
            tot += w[n] * orc.kinetic_y(p, f)[0]
        return tot

    fs = [f0]
    for n in range(N):
        fs.append(orc.step(p, fs[-1]))
    lam = w[N] * orc.kinetic_y_grad(p, fs[N])
    for n in range(N - 1, -1, -1):
        lam = orc.adjoint_step(p, fs[n], lam, w[n])
    d = inputs.random_like(f0.shape, 9, scale=f0.std())
    fd = _fd(J, f0, d)
    assert np.sum(lam * d) == pytest.approx(fd, rel=1e-7)
