"""The C ABI from plain C: tests/c/c_abi_check.c (built by
__graft_entry__.build() into paper_2311_14941_amd/_build/) loads the
9-species mechanism, integrates 64 cells held in hipMalloc'd buffers with
default options and writes the results; they must equal the Python
binding's bit for bit (same library, same kernels)."""
import os
import subprocess

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2311_14941_amd", "_build", "c_abi_check")


def test_c_program_matches_python_binding(tmp_path):
    import torch
    import paper_2311_14941_amd as sc
    from synth.cells import make_cells
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    assert os.path.exists(EXE), "c_abi_check is built by __graft_entry__.build()"
    sc.ensure_built()
    c = make_cells("C1", n=64)
    text = c["mech"].to_text()
    n, N = c["T"].size, c["mech"].n_species
    mech_path, inp, outp = tmp_path / "mech.txt", tmp_path / "in.bin", tmp_path / "out.bin"
    mech_path.write_text(text)
    Ysm = np.ascontiguousarray(c["Y"].T)  # species-major
    with open(inp, "wb") as f:
        f.write(np.int64(n).tobytes())
        for a in (c["T"], c["p"], Ysm, c["dt"]):
            f.write(np.ascontiguousarray(a, np.float64).tobytes())
    print("running", EXE, flush=True)
    r = subprocess.run([EXE, str(mech_path), str(inp), str(outp)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    raw = outp.read_bytes()
    nd = n * (N + 1)
    vals = np.frombuffer(raw[:8 * nd], np.float64)
    ints = np.frombuffer(raw[8 * nd:], np.int32)
    T1c, Y1c = vals[:n], vals[n:].reshape(N, n)
    stc, nac = ints[:n], ints[n:]
    d = "cuda:0"
    plan = sc.Plan(sc.Mechanism(text))
    out = plan.integrate(torch.tensor(c["T"], device=d), torch.tensor(c["p"], device=d),
                         torch.tensor(Ysm, device=d), torch.tensor(c["dt"], device=d))
    assert np.all(stc == 0)
    assert np.array_equal(T1c, out["T"].cpu().numpy())
    assert np.array_equal(Y1c, out["Y"].cpu().numpy())
    assert np.array_equal(nac, out["n_acc"].cpu().numpy())
