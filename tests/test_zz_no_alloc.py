"""The allocation-free integration entry point (sc_integrate_noalloc) against
sc_integrate, through the C ABI: same kernels, so results must agree bit for
bit, on two calls in a row (the second with fewer cells, so the shared fixed
scratch holds the first call's contents), in every launch mode and cell
order, and the cell limit is refused before any launch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a HIP device"
    return t


@pytest.fixture(scope="module")
def sc():
    import paper_2311_14941_amd as m
    m.ensure_built()
    return m


@pytest.fixture(scope="module")
def c2():
    from synth.cells import make_cells
    return make_cells("C2")


def _gpu(torch, c, idx):
    d = "cuda:0"
    return (torch.tensor(c["T"][idx], device=d), torch.tensor(c["p"][idx], device=d),
            torch.tensor(np.ascontiguousarray(c["Y"][idx].T), device=d), torch.tensor(c["dt"][idx], device=d))


def _out(torch, T, Y, na, nr):
    n = T.shape[0]
    return dict(T=torch.empty_like(T), Y=torch.empty_like(Y),
                status=torch.empty(n, dtype=torch.int32, device=T.device), n_acc=na.clone(), n_rej=nr.clone())


@pytest.mark.parametrize("mode,order", [("persistent", "cost"), ("persistent", "dt"), ("persistent", "none"),
                                        ("plain", "none"), ("static", "none")])
def test_noalloc_matches_integrate_two_calls(torch, sc, c2, mode, order):
    mech = sc.Mechanism(c2["mech"].to_text())
    plan = sc.Plan(mech, rtol=1e-6, atol=1e-12, mode=mode, order=order)
    rng = np.random.default_rng(3)
    for n in (20000, 3001):  # second call smaller: the scratch keeps the first call's contents
        idx = np.sort(rng.choice(c2["T"].size, n, replace=False))
        T, p, Y, dt = _gpu(torch, c2, idx)
        # predicted costs for the cost order: a previous integration's counts
        prev = sc.Plan(mech, rtol=1e-6, atol=1e-12).integrate(T, p, Y, dt)
        ref = plan.integrate(T, p, Y, dt, out=_out(torch, T, Y, prev["n_acc"], prev["n_rej"]))
        got = plan.integrate_noalloc(T, p, Y, dt, out=_out(torch, T, Y, prev["n_acc"], prev["n_rej"]))
        torch.cuda.synchronize()
        for k in ("T", "Y", "status", "n_acc", "n_rej"):
            assert torch.equal(ref[k], got[k]), (mode, order, n, k)
        assert bool((got["status"] == 0).all())


def test_noalloc_with_carried_step_and_no_device_allocation(torch, sc, c2):
    """Carried step sizes (h in, next h out) agree bit for bit too; the call
    leaves the device's free memory unchanged (nothing allocated)."""
    mech = sc.Mechanism(c2["mech"].to_text())
    idx = np.arange(0, 65536, 7)[:8192]
    T, p, Y, dt = _gpu(torch, c2, idx)
    h0 = dt * 1e-3
    plan = sc.Plan(mech, mode="persistent", order="dt")
    ref = plan.integrate(T, p, Y, dt, h=h0)
    fresh = sc.Plan(mech, mode="persistent", order="dt")
    out = _out(torch, T, Y, torch.zeros_like(ref["n_acc"]), torch.zeros_like(ref["n_rej"]))
    hio = h0.clone()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    got = fresh.integrate_noalloc(T, p, Y, dt, h=hio, out=out)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    for k in ("T", "Y", "status", "n_acc", "n_rej", "h"):
        assert torch.equal(ref[k], got[k]), k
    assert free1 == free0


def test_noalloc_refuses_more_cells_than_its_scratch(torch, sc, c2):
    mech = sc.Mechanism(c2["mech"].to_text())
    plan = sc.Plan(mech, mode="persistent", order="cost")
    n = 262145
    idx = np.arange(n) % c2["T"].size
    T, p, Y, dt = _gpu(torch, c2, idx)
    with pytest.raises(sc.StiffchemError) as e:
        plan.integrate_noalloc(T, p, Y, dt)
    assert e.value.code == sc.SC_EINVAL and "262144" in str(e.value)
