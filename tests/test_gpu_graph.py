"""A whole step (neighbour build + energy/forces/virial) captured once into a
HIP graph and replayed: every replay, on moved positions, must match an
eager evaluation of the same positions bit for bit, and the oracle to the
parity tolerances.  Eager work on other streams and host synchronisations
run between the replays.
"""

import numpy as np
import pytest

import synth
from oracle import d3_ref as R

pytestmark = pytest.mark.gpu

TAB = synth.make_table()


def _capture(calc, system, out, build, stream):
    import torch
    from paper_2310_05279_amd import d3
    cell = np.ascontiguousarray(system["cell"], dtype=np.float64)
    pbc = np.ascontiguousarray(system["pbc"], dtype=np.int32)

    def step():
        if build == "call":
            d3.d3_build_neighbors(calc.ctx, calc.pos, calc.types, cell, pbc, stream)
        flags = d3.D3_REBUILD if build == "flag" else 0
        d3.d3_energy_forces_virial(calc.ctx, calc.pos, out["energy"], out["forces"],
                                   out["virial"], out["atom_energy"], flags, stream)

    with torch.cuda.stream(stream):
        for _ in range(3):
            step()
    torch.cuda.synchronize()
    calc.status()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        step()
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("mode,build,skin,scale", [
    ("plain", "call", 0.0, 0.05),
    ("prec", "call", 0.0, 0.05),
    ("plain", "flag", 0.0, 0.05),
    ("plain", None, 1.0, 0.1),
])
def test_graph_replays_match_eager(mode, build, skin, scale):
    import torch
    from paper_2310_05279_amd import d3
    m = synth.mof_like(3000, seed=77)
    n = m["pos"].shape[0]
    print("graph case mode=%s build=%s skin=%.1f n=%d" % (mode, build, skin, n), flush=True)
    calc = d3.D3(TAB, mode=mode, skin=skin)
    calc.build(m["pos"], m["types"], m["cell"], m["pbc"])
    dev = torch.device("cuda", 0)
    out = {"energy": torch.zeros(1, dtype=torch.float64, device=dev),
           "forces": torch.zeros((n, 3), dtype=torch.float64, device=dev),
           "virial": torch.zeros((3, 3), dtype=torch.float64, device=dev),
           "atom_energy": torch.zeros(n, dtype=torch.float64, device=dev)}
    s = torch.cuda.Stream()
    g = _capture(calc, m, out, build, s)
    ref = d3.D3(TAB, mode=mode, skin=skin)
    if not build:
        # lists kept from the first build: the eager run keeps the same lists
        ref.build(m["pos"], m["types"], m["cell"], m["pbc"])
    rng = np.random.default_rng(5)
    base = calc.pos.clone()
    junk = torch.zeros(1 << 20, dtype=torch.float64, device=dev)
    for rep in range(4):
        disp = rng.uniform(-scale, scale, size=(n, 3))
        calc.pos.copy_(base + torch.as_tensor(disp, device=dev))
        junk.add_(1.0)                       # unrelated eager work on the default stream
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        calc.status()
        pos = calc.pos.cpu().numpy()
        if build:
            ref.build(pos, m["types"], m["cell"], m["pbc"])
        o = ref.compute(pos)
        torch.cuda.synchronize()
        for k in ("energy", "forces", "virial", "atom_energy"):
            assert torch.equal(out[k], o[k]), "replay %d: %s differs from eager" % (rep, k)
        if rep == 1 and mode == "plain":
            r = R.d3(pos, m["types"], m["cell"], m["pbc"], TAB)
            de = abs(float(out["energy"][0]) - r["energy"]) / n
            df = np.abs(out["forces"].cpu().numpy() - r["forces"]).max()
            print("replay %d vs oracle |dE|/atom=%.2e max|dF|=%.2e" % (rep, de, df), flush=True)
            assert de <= 1e-6 and df <= 1e-5
        print("replay %d bitwise equal to eager" % rep, flush=True)
    assert float(junk[0]) == 4.0
    del g
    ref.close()
    calc.close()
