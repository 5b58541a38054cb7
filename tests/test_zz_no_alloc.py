"""dg_rk_step_noalloc: the RK step whose stage states live in the library's
per-GPU scratch array, called through the C ABI and compared with dg_rk_step
(caller work buffer) on the same inputs.  Both run the same stage kernels in
the same order, so the results must agree bit for bit (stricter than the
parity bar).  Two calls in a row on one GPU share the scratch array; the
second uses a smaller mesh.  A mesh whose stage states exceed the scratch is
refused before anything is enqueued."""
import ctypes
import sys

import numpy as np
import pytest

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


def _noalloc(dg, mesh, q, dt, scheme, nsteps):
    lib = dg._lib.load()
    return lib.dg_rk_step_noalloc(mesh._ctx, ctypes.c_void_p(q.data_ptr()), ctypes.c_double(dt),
                                  ctypes.c_int32(scheme), ctypes.c_int32(nsteps), None)


def _compare(dg, n_lon, n_lat, order, dtype, scheme, nsteps, lmax, seed):
    from dg_inputs import band_limited_state
    qh, info = band_limited_state(n_lon, n_lat, order, lmax, seed)
    mesh = dg.Mesh(n_lon, n_lat, order, dtype=dtype)
    q0 = torch.from_numpy(qh).to("cuda", mesh.dtype)
    dt = dg.cfl_time_step(mesh, info.cmax, 0.1)
    ref = q0.clone()
    mesh.rk_step(ref, mesh.empty_work(scheme), dt, scheme=scheme, nsteps=nsteps)
    got = q0.clone()
    rc = _noalloc(dg, mesh, got, dt, scheme, nsteps)
    assert rc == 0, dg._lib.load().dg_last_error()
    torch.cuda.synchronize()
    diff = (got - ref).abs().max().item()
    say("noalloc", n_lon, n_lat, order, dtype, "scheme", scheme, "steps", nsteps, "max diff", diff)
    assert torch.equal(got, ref)
    assert np.all(np.isfinite(got.cpu().numpy()))


def test_noalloc_matches_rk_step_twice_second_smaller(dg):
    # first call: the 180 x 90 r = 3 FP64 workload, SSP-RK3 (12.4 MB of stage states)
    _compare(dg, 180, 90, 3, "f64", dg.DG_SSP_RK3, 3, 16, 2)
    # second call on the same scratch, smaller mesh: 32 x 16 r = 1
    _compare(dg, 32, 16, 1, "f64", dg.DG_SSP_RK3, 5, 6, 1)


def test_noalloc_rk4_and_f32(dg):
    # RK4 at the largest state that fits (3 states, 18.7 MB), then FP32 RK2
    _compare(dg, 180, 90, 3, "f64", dg.DG_RK4, 2, 16, 2)
    _compare(dg, 90, 45, 2, "f32", dg.DG_SSP_RK2, 4, 16, 3)


def test_noalloc_refuses_states_beyond_scratch(dg):
    lib = dg._lib.load()
    mesh = dg.Mesh(360, 180, 5, dtype="f32")        # RK3 stage states: 56 MB > 32 MiB
    q = torch.ones(mesh.state_size(), dtype=mesh.dtype, device="cuda")
    before = q.clone()
    rc = _noalloc(dg, mesh, q, 1.0, dg.DG_SSP_RK3, 1)
    msg = lib.dg_last_error().decode()
    say("refusal", rc, msg)
    assert rc == dg._lib.DG_EINVAL
    assert "scratch" in msg
    torch.cuda.synchronize()
    assert torch.equal(q, before)
