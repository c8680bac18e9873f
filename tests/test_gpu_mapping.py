"""Parity of the zonal reference-cell mapping (sc_plan_set_mapping,
sc_integrate_mapped) against its CPU reference (oracle/mapping.py) on the
flame's mixing-layer cells (synth.field.mixing_cells): the reference of
every cell bit for bit, the integrated and the mapped cells' states within
the parity bar at rtol 1e-10 against the oracle at rtol 1e-11, step counts
and status of mapped cells, launch modes bit for bit, a bound below every
cell equal to sc_integrate bit for bit, and the argument errors."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

Z_TOL, DT_BAND = 1e-3, 2.0


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
def cells():
    from synth.field import mixing_cells
    return mixing_cells()


@pytest.fixture(scope="module")
def ref_oracle(cells):
    from oracle import mapping as om
    from oracle.oracle import Oracle
    text = cells["mech"].to_text()
    return om.integrate_mapped(Oracle(text), text, cells["T"], cells["p"], cells["Y"], cells["dt"],
                               cells["Y_fuel"], cells["Y_ox"], Z_TOL, DT_BAND, rtol=1e-11, atol=1e-17,
                               max_steps=200000)


def _gpu(torch, c):
    d = "cuda:0"
    return (torch.tensor(c["T"], device=d), torch.tensor(c["p"], device=d),
            torch.tensor(np.ascontiguousarray(c["Y"].T), device=d), torch.tensor(c["dt"], device=d))


def _plan(sc, c, **kw):
    plan = sc.Plan(sc.Mechanism(c["mech"].to_text()), **kw)
    plan.set_mapping(c["Y_fuel"], c["Y_ox"], Z_TOL, DT_BAND)
    return plan


@pytest.mark.parametrize("linalg", ["dense", "sparse"])
def test_mapping_parity(torch, sc, cells, ref_oracle, linalg):
    plan = _plan(sc, cells, rtol=1e-10, atol=1e-16, max_steps=200000, linalg=linalg)
    T, p, Y, dt = _gpu(torch, cells)
    r = plan.integrate_mapped(T, p, Y, dt)
    ref = r["ref"].cpu().numpy()
    assert np.array_equal(ref, ref_oracle["ref"])
    mapped = ref != np.arange(ref.size)
    assert mapped.sum() > 100 and (~mapped).sum() > 100
    assert np.all(r["status"].cpu().numpy() == 0)
    assert np.all(r["n_acc"].cpu().numpy()[mapped] == 0) and np.all(r["n_rej"].cpu().numpy()[mapped] == 0)
    assert np.all(r["n_acc"].cpu().numpy()[~mapped] > 0)
    T1, Y1 = r["T"].cpu().numpy(), r["Y"].cpu().numpy().T
    Tr, Yr = ref_oracle["T"], ref_oracle["Y"]
    assert np.all(np.abs(T1 - Tr) <= 1e-6 * Tr)
    big = np.abs(Yr) > 1e-8
    assert np.all(np.abs(Y1 - Yr)[big] <= 1e-6 * np.abs(Yr)[big])
    assert np.all(np.abs(Y1 - Yr)[~big] <= 1e-12)


def test_mapping_launch_modes_bitwise(torch, sc, cells):
    T, p, Y, dt = _gpu(torch, cells)
    outs = []
    for kw in (dict(mode="plain"), dict(mode="static"), dict(mode="persistent", order="cost")):
        plan = _plan(sc, cells, **kw)
        r = plan.integrate_mapped(T, p, Y, dt)
        if kw.get("order") == "cost":
            r = plan.integrate_mapped(T, p, Y, dt, out=r)
        outs.append(r)
    for r in outs[1:]:
        for k in ("T", "Y", "status", "n_acc", "n_rej", "ref"):
            assert torch.equal(r[k], outs[0][k]), k


def test_mapping_nothing_mapped_equals_integrate(torch, sc, cells):
    """With a bound below every cell's mixture fraction no cell is mapped:
    the result is sc_integrate's bit for bit."""
    T, p, Y, dt = _gpu(torch, cells)
    plan = sc.Plan(sc.Mechanism(cells["mech"].to_text()))
    plan.set_mapping(cells["Y_fuel"], cells["Y_ox"], -1e300, DT_BAND)
    a = plan.integrate(T, p, Y, dt)
    b = plan.integrate_mapped(T, p, Y, dt)
    assert np.array_equal(b["ref"].cpu().numpy(), np.arange(T.numel()))
    for k in ("T", "Y", "status", "n_acc", "n_rej"):
        assert torch.equal(a[k], b[k]), k


def test_mapping_arguments(torch, sc, cells):
    T, p, Y, dt = _gpu(torch, cells)
    plan = sc.Plan(sc.Mechanism(cells["mech"].to_text()))
    with pytest.raises(RuntimeError, match="set_mapping"):
        plan.integrate_mapped(T, p, Y, dt)
    with pytest.raises(RuntimeError, match="dT"):
        plan.set_mapping(cells["Y_fuel"], cells["Y_ox"], Z_TOL, 0.0)
    with pytest.raises(RuntimeError, match="same coupling"):
        plan.set_mapping(cells["Y_ox"], cells["Y_ox"], Z_TOL, DT_BAND)
    with pytest.raises(RuntimeError, match="zones"):
        plan.set_mapping(cells["Y_fuel"], cells["Y_ox"], Z_TOL, 1e-4, 1e-4)
    plan.set_mapping(cells["Y_fuel"], cells["Y_ox"], Z_TOL, DT_BAND)
    out = dict(T=T, Y=Y, status=torch.empty(T.numel(), dtype=torch.int32, device=T.device),
               n_acc=torch.zeros(T.numel(), dtype=torch.int32, device=T.device),
               n_rej=torch.zeros(T.numel(), dtype=torch.int32, device=T.device))
    with pytest.raises(RuntimeError, match="apart"):
        plan.integrate_mapped(T, p, Y, dt, out=out)
