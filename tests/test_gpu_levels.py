"""Identical vertical layers (section 5.2.2: decoupled two-dimensional problems
solved side by side) through dg_set_levels: every layer of a multi-layer
state gives the oracle's right-hand side, and the same bits as the
one-layer context on that layer alone (the layers share the kernel and its
summation order); RK steps, the graph path and the mass diagnostic follow;
the calls defined for one layer reject more."""
import sys

import numpy as np
import pytest

from dg_inputs import band_limited_state, random_plane_state
from oracle import PlaneDG, SphereDG
from parity_util import TOL, errors

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_11767_amd as dg
    return dg


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def td(dtype):
    return torch.float64 if dtype == "f64" else torch.float32


def layers(n_lon, n_lat, order, nz, seed0):
    """nz different seeded states of one mesh, stacked [nz][E][3][N]."""
    qs = [band_limited_state(n_lon, n_lat, order, 4, seed0 + k)[0] for k in range(nz)]
    return np.stack(qs)


@pytest.mark.parametrize("kernel", ["line", "half"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("order", [1, 3, 4])
def test_layers_rhs_match_oracle_and_single_layer(dg, kernel, dtype, order):
    nl, nt, nz = 13, 7, 3
    say("levels rhs", nl, nt, order, dtype, kernel, nz)
    q = layers(nl, nt, order, nz, 300 + order)
    mesh = dg.Mesh(nl, nt, order, dtype=dtype, h_ref=1e4 if dtype == "f32" else 0.0)
    mesh.kernel = kernel
    one = [mesh.rhs(torch.from_numpy(q[k]).to("cuda", td(dtype))).cpu() for k in range(nz)]
    mesh.levels = nz
    assert mesh.levels == nz and mesh.state_size() == nz * mesh.E * 3 * mesh.N
    got = mesh.rhs(torch.from_numpy(q).to("cuda", td(dtype))).cpu()
    assert got.shape == (nz, mesh.E, 3, mesh.N)
    m = SphereDG(nl, nt, order)
    for k in range(nz):
        assert torch.equal(got[k], one[k]), k
        qin = q[k].astype(np.float32).astype(np.float64) if dtype == "f32" else q[k]
        comp, norm = errors(got[k].numpy(), m.rhs(qin), m.rhs_scale(qin))
        say("  layer", k, "componentwise", comp)
        assert np.all(comp <= TOL[dtype]), (k, comp)


@pytest.mark.parametrize("scheme", ["rk3", "rk4"])
def test_layers_rk_steps_and_mass(dg, scheme):
    nl, nt, order, nz = 16, 8, 2, 4
    say("levels steps", nl, nt, order, nz, scheme)
    sch = dg.DG_SSP_RK3 if scheme == "rk3" else dg.DG_RK4
    q = layers(nl, nt, order, nz, 400)
    mesh = dg.Mesh(nl, nt, order)
    singles = []
    mass1 = np.zeros(3)
    for k in range(nz):
        qk = torch.from_numpy(q[k]).to("cuda")
        mesh.rk_step(qk, mesh.empty_work(sch), 30.0, scheme=sch, nsteps=5)
        singles.append(qk.cpu())
        mass1 += np.array(mesh.mass(qk))
    mesh.levels = nz
    qa = torch.from_numpy(q).to("cuda")
    mesh.rk_step(qa, mesh.empty_work(sch), 30.0, scheme=sch, nsteps=5)
    for k in range(nz):
        assert torch.equal(qa[k].cpu(), singles[k]), k
    mass = np.array(mesh.mass(qa))
    assert np.allclose(mass, mass1, rtol=1e-13, atol=1e-13 * np.abs(mass1).max())


def test_layers_graph_replay(dg):
    nl, nt, order, nz = 12, 6, 3, 5
    say("levels graph", nl, nt, order, nz)
    q = layers(nl, nt, order, nz, 500)
    mesh = dg.Mesh(nl, nt, order)
    mesh.levels = nz
    qe = torch.from_numpy(q).to("cuda")
    mesh.rk_step(qe, mesh.empty_work(), 40.0, nsteps=6)
    qg = torch.from_numpy(q).to("cuda")
    w = mesh.empty_work()
    g = mesh.graph(qg, w, 40.0, nsteps=2)
    for _ in range(3):
        g.launch()
        torch.cuda.synchronize()
    g.close()
    assert torch.equal(qe, qg)


def test_plane_layers_match_oracle(dg):
    nx, ny, order, nz = 9, 5, 3, 2
    say("plane levels", nx, ny, order, nz)
    lx, ly = 1e7, 0.8e7
    q = np.stack([random_plane_state(nx, ny, order, lx, ly, 600 + k) for k in range(nz)])
    mesh = dg.Plane(nx, ny, order, lx, ly, f=1e-4, gravity=9.81)
    mesh.levels = nz
    got = mesh.rhs(torch.from_numpy(q).to("cuda")).cpu().numpy()
    m = PlaneDG(nx, ny, order, lx, ly, gravity=9.81, f=1e-4)
    for k in range(nz):
        comp, _ = errors(got[k], m.rhs(q[k]), m.rhs_scale(q[k]))
        assert np.all(comp <= TOL["f64"]), (k, comp)


def test_levels_argument_checks(dg):
    mesh = dg.Mesh(8, 4, 1)
    for bad in (0, -2, 65536):
        with pytest.raises(dg.DGError):
            mesh.levels = bad
    assert mesh.levels == 1
    mesh.levels = 2
    with pytest.raises(ValueError):        # a one-layer buffer no longer fits
        mesh.rhs(torch.zeros((mesh.E, 3, mesh.N), dtype=torch.float64, device="cuda"))
    # the learned calls are defined for one layer
    import ctypes
    q = mesh.empty_state()
    X = torch.empty((mesh.E, 108), dtype=torch.float32, device="cuda")
    rc = mesh._lib.dg_features(mesh._ctx, ctypes.c_void_p(q.data_ptr()), None, None,
                               ctypes.c_void_p(X.data_ptr()), None)
    assert rc == -6
    mesh.levels = 1
    ens = dg.Ensemble([dict(n_lon=8, n_lat=4, order=1), dict(n_lon=6, n_lat=3, order=2)])
    with pytest.raises(dg.DGError):
        ens.members[0].levels = 2
    assert ens.members[0].levels == 1


@pytest.mark.parametrize("kernel", ["line", "half"])
def test_layers_in_multiwave_workgroups(dg, kernel):
    """180 x 90, r = 3 with 5 layers: enough wavefronts for the launch shape
    of four wavefronts per workgroup (and, for the half layout, elements
    packed across row ends); every layer equals the one-layer result, which
    is itself checked against the oracle at this mesh."""
    nl, nt, order, nz = 180, 90, 3, 5
    say("levels multiwave", nl, nt, order, nz, kernel)
    qa = band_limited_state(nl, nt, order, 16, 2)[0]
    qb = band_limited_state(nl, nt, order, 8, 7)[0]
    q = np.stack([qa, qb, qa, qb, qa])
    mesh = dg.Mesh(nl, nt, order)
    mesh.kernel = kernel
    one = [mesh.rhs(torch.from_numpy(x).to("cuda")).cpu() for x in (qa, qb)]
    mesh.levels = nz
    got = mesh.rhs(torch.from_numpy(q).to("cuda")).cpu()
    for k in range(nz):
        assert torch.equal(got[k], one[k % 2]), k


def test_autotune_with_layers(dg):
    """dg_autotune on a three-layer state: reads it only, keeps a layout, and
    the layers still agree bitwise with one-layer runs of that layout."""
    nl, nt, order, nz = 40, 20, 3, 3
    say("levels autotune", nl, nt, order, nz)
    q = layers(nl, nt, order, nz, 800)
    mesh = dg.Mesh(nl, nt, order)
    mesh.levels = nz
    qd = torch.from_numpy(q).to("cuda")
    before = qd.clone()
    name = mesh.autotune(qd)
    assert torch.equal(qd, before) and mesh.kernel == name
    got = mesh.rhs(qd).cpu()
    single = dg.Mesh(nl, nt, order)
    single.kernel = name
    for k in range(nz):
        assert torch.equal(got[k], single.rhs(torch.from_numpy(q[k]).to("cuda")).cpu()), k
