"""Convergence of the whole GPU path on a manufactured steady state.

A smooth state U* on the sphere is made steady by the forcing
f = dF/dlam + dG/dtheta - S of U* (its modal weak projection set with
dg_set_forcing); the GPU then runs SSP-RK3 from the projection of U* for one
simulated hour, and the cos-weighted L2 error of h against the projection
of U* is measured on three meshes per order.  The paper's convergence
tables report order about r + 1 for smooth solutions (2.00 / 3.00 /
3.96-4.00 for p = 1, 2, 3); the test asserts the finest-pair rate within
0.3 of r + 1 for r = 1..5 (r = 5: the order of the 360 x 180 FP32
workload).  Forcing and projections come from the oracle (inputs only); the
run is the library's."""
import sys

import numpy as np
import pytest

from oracle import SphereDG

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

R, G, OM = 6.371e6, 9.80616, 7.292e-5
H0 = 1e4


@pytest.fixture(scope="module")
def dg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_11767_amd as dg
    return dg


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _fields(lam, th):
    h = H0 + 100 * np.cos(th) ** 2 * np.sin(lam) + 50 * np.sin(th) * np.cos(th)
    u = 20 * np.cos(th) + 5 * np.sin(2 * lam) * np.cos(th) ** 2
    v = 8 * np.cos(lam) * np.cos(th) ** 2 * np.sin(th)
    return h, u, v


def _q_exact(lam, th):
    h, u, v = _fields(lam, th)
    return np.array([h, h * u, h * v])


def _forcing_density(lam, th):
    """dF/dlam + dG/dtheta - S of the fields (complex-step derivatives)."""
    eps = 1e-30

    def FG(l, t):
        h, u, v = _fields(l, t)
        p = 0.5 * G * h * h
        return (np.array([h * u, h * u * u + p, h * u * v]) / R,
                np.cos(t) * np.array([h * v, h * u * v, h * v * v + p]) / R)

    dF = FG(lam + 1j * eps, th + 0j)[0].imag / eps
    dG = FG(lam + 0j, th + 1j * eps)[1].imag / eps
    h, u, v = _fields(lam, th)
    p = 0.5 * G * h * h
    cor = 2 * OM * np.sin(th) * np.cos(th) + u * np.sin(th) / R
    S = np.array([0 * h, cor * h * v, -p * np.sin(th) / R - cor * h * u])
    return dF + dG - S


def _h_error(m, q, ref):
    d = m.grid(q - ref)[:, :, 0]                       # [j, i, N]
    r = m.grid(ref)[:, :, 0]
    e2 = np.einsum("jim,jmn,jin->", d, m.M, d)
    n2 = np.einsum("jim,jmn,jin->", r, m.M, r)
    return np.sqrt(e2 / n2)


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5])
def test_manufactured_steady_state_converges(dg, order):
    errs = []
    for n_lat in (8, 16, 32):
        n_lon = 2 * n_lat
        m = SphereDG(n_lon, n_lat, order)
        q0 = np.ascontiguousarray(m.project(_q_exact))
        f = m.weak_forcing(_forcing_density)
        mesh = dg.Mesh(n_lon, n_lat, order, dtype="f64")
        qd = torch.from_numpy(q0).cuda()
        fd = torch.from_numpy(np.ascontiguousarray(f)).cuda()
        mesh.set_forcing(fd)
        dt = dg.cfl_time_step(mesh, 20.0 + np.sqrt(G * (H0 + 150.0)) + 10.0, 0.05)
        steps = int(np.ceil(3600.0 / dt))
        mesh.rk_step(qd, mesh.empty_work(), 3600.0 / steps, nsteps=steps)
        mesh.set_forcing(None)
        err = _h_error(m, qd.cpu().numpy(), q0)
        say("mms", order, n_lon, n_lat, "steps", steps, "h error", err)
        errs.append(err)
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    say("  rates", rates)
    assert np.all(np.isfinite(errs))
    assert abs(rates[-1] - (order + 1)) < 0.3, (errs, rates)
