"""MD checkpoint and resume through the C ABI: 100 + 100 steps with a
checkpoint in between, in a fresh context, give the same bits as 200 steps
in one run (positions, velocities, energies and the rebuild count)."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TAB = synth.make_table()


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    return torch


def test_build_positions_are_the_callers_exactly():
    """The build positions come back bit for bit, in the caller's order,
    unwrapped, also for atoms given far outside the cell."""
    torch = _torch()
    from paper_2310_05279_amd import d3
    m = synth.mof_like(800, seed=21)
    rng = np.random.default_rng(21)
    pos = m["pos"] + rng.integers(-3, 4, (800, 1)) * m["cell"][0] \
        + rng.integers(-2, 3, (800, 1)) * m["cell"][2]
    calc = d3.D3(TAB, skin=1.0)
    calc.build(pos, m["types"], m["cell"], m["pbc"])
    out = torch.full((800, 3), float("nan"), dtype=torch.float64, device="cuda")
    d3.d3_build_positions(calc.ctx, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), pos)
    calc.close()


@pytest.mark.parametrize("mode", ["plain", "prec"])
def test_md_resume_is_bitwise(tmp_path, mode):
    """200 steps in one run against a checkpoint near step 100 (the first
    step from 100 on that falls between two list builds) and a resumed run
    in a new context: the same bits, the same energies at every step and
    the same number of builds."""
    torch = _torch()
    from paper_2310_05279_amd import d3, md_state
    m = synth.mof_like(2000, seed=12)
    vel, mass = synth.maxwell_velocities(m["types"], 300.0, seed=301)
    ms = torch.as_tensor(mass, device="cuda")
    types = torch.as_tensor(m["types"], dtype=torch.int32, device="cuda")
    total = 200

    def fresh():
        calc = d3.D3(TAB, mode=mode, skin=1.0)
        calc.build(m["pos"], m["types"], m["cell"], m["pbc"])
        p = torch.as_tensor(m["pos"], device="cuda").clone()
        v = torch.as_tensor(vel, device="cuda").clone()
        return calc, p, v

    # one run of 200 steps, energies recorded at every step
    a, pa, va = fresh()
    th_a, reb_a = d3.d3_md_nve(a.ctx, total, 1.0, pa, va, ms, every=1)
    # 100 steps, then single steps until the lists were built at an earlier
    # step than the current one; a checkpoint there; the context closed
    b, pb, vb = fresh()
    _, reb_b = d3.d3_md_nve(b.ctx, 100, 1.0, pb, vb, ms)
    k = 100
    bp = torch.empty_like(pb)
    while True:
        d3.d3_build_positions(b.ctx, bp)
        torch.cuda.synchronize()
        if not torch.equal(bp, pb) or k >= 130:
            break
        _, r = d3.d3_md_nve(b.ctx, 1, 1.0, pb, vb, ms)
        reb_b += r
        k += 1
    path = str(tmp_path / "md.npz")
    md_state.save(path, b.ctx, pb, vb, k)
    b.close()
    st = md_state.load(path)
    assert st["step"] == k
    assert not np.array_equal(st["build_pos"], st["pos"])
    # resumed in a new context for the remaining steps
    c = d3.D3(TAB, mode=mode, skin=1.0)
    pc, vc = md_state.resume(c.ctx, st, types, m["cell"], m["pbc"])
    th_c, reb_c = d3.d3_md_nve(c.ctx, total - k, 1.0, pc, vc, ms, every=1)
    torch.cuda.synchronize()
    print("resume %s at step %d: builds %d = %d + %d, max|dx| %.1e"
          % (mode, k, reb_a, reb_b, reb_c, (pa - pc).abs().max().item()), flush=True)
    assert 5 <= reb_a <= 60 and reb_c >= 1
    assert reb_a == reb_b + reb_c
    assert torch.equal(pa, pc) and torch.equal(va, vc)
    assert np.array_equal(th_a[k:], th_c)
    a.close()
    c.close()
