"""Per-atom virial (Eq. 7) and heat current (Eq. 8) of the HIP path, through
the C ABI's d3_evaluate, against the FP64 oracle.

Gates: plain FP64, max |dW_i| <= 1e-9 max |W_i| and the same for J_i;
precision form, max |dW_i| <= 1e-5 eV.  Asking for the per-atom outputs
must not change any other output (bitwise), and sum_i W_i must equal the
virial.
"""

import numpy as np
import pytest

import synth
from oracle import d3_oracle as O
from oracle import d3_ref as R

pytestmark = pytest.mark.gpu

TAB = synth.make_table()


def _tiny():
    cell = np.array([[5.0, 0.0, 0.0], [2.0, 4.6, 0.0], [0.5, 0.7, 5.3]])
    frac = np.random.default_rng(2).uniform(0, 1, (4, 3))
    return {"pos": frac @ cell, "types": np.array([0, 1, 2, 4], np.int32), "cell": cell,
            "pbc": np.array([1, 1, 1], np.int32)}


def _system(case):
    if case == "graphene144":
        return synth.bilayer_graphene(), O
    if case == "tiny":
        return _tiny(), O
    return synth.mof_like(3000, seed=31), R


def _run(s, mode, vel, prep=None, **prm):
    import torch
    from paper_2310_05279_amd import d3
    calc = d3.D3(TAB, mode=mode, **prm)
    calc.build(s["pos"], s["types"], s["cell"], s["pbc"])
    if prep:
        prep(calc)
    base = calc.compute()
    full = calc.compute(atom_virial=True, velocities=vel)
    torch.cuda.synchronize()
    calc.status()
    for k in ("energy", "forces", "virial", "atom_energy"):
        assert torch.equal(base[k], full[k]), "%s changed when per-atom virials were asked" % k
    out = {k: v.cpu().numpy() for k, v in full.items() if v is not None}
    calc.close()
    return out


def _sum_rule(out):
    W = out["virial"]
    s = out["atom_virial"].sum(0)
    assert np.abs(s - W).max() <= 1e-11 * np.abs(W).max()


@pytest.mark.parametrize("case", ["graphene144", "tiny", "mof3000"])
def test_atom_virial_and_heat_current_plain(case):
    s, oracle = _system(case)
    n = s["pos"].shape[0]
    print("atom virial case", case, n, flush=True)
    vel = np.random.default_rng(9).normal(scale=0.01, size=(n, 3))
    ref = oracle.d3(s["pos"], s["types"], s["cell"], s["pbc"], TAB)
    out = _run(s, "plain", vel)
    W, Wr = out["atom_virial"], ref["atom_virial"]
    J, Jr = out["heat_current"], O.heat_current(Wr, vel)
    dw = np.abs(W - Wr).max() / np.abs(Wr).max()
    dj = np.abs(J - Jr).max() / np.abs(Jr).max()
    print("%s max|dW_i|/max|W_i| = %.2e, max|dJ_i|/max|J_i| = %.2e" % (case, dw, dj), flush=True)
    assert dw <= 1e-9 and dj <= 1e-9
    assert np.abs(W - W.transpose(0, 2, 1)).max() == 0.0
    _sum_rule(out)


@pytest.mark.parametrize("mode,variant", [("plain", "zero"), ("literal", "bj"),
                                          ("literal", "zero_atm")])
def test_atom_virial_variants_and_literal_mode(mode, variant):
    """The per-atom virial and heat current with zero damping (and the
    three-body term), and in the mode that sums Eq. 3 as printed: against
    the oracle, on a 1 200-atom MOF-like cell, with the same gates as the
    plain form."""
    zero = dict(damping="zero", s8=0.722, rs6=1.217, rs8=1.0)
    prm = {"bj": {}, "zero": zero, "zero_atm": dict(zero, s9=1.0)}[variant]
    s = synth.mof_like(1200, seed=36)
    n = s["pos"].shape[0]
    vel = np.random.default_rng(10).normal(scale=0.01, size=(n, 3))
    ref = O.d3(s["pos"], s["types"], s["cell"], s["pbc"], TAB, O.Params(**prm))
    out = _run(s, mode, vel, **prm)
    W, Wr = out["atom_virial"], ref["atom_virial"]
    J, Jr = out["heat_current"], O.heat_current(Wr, vel)
    dw = np.abs(W - Wr).max() / np.abs(Wr).max()
    dj = np.abs(J - Jr).max() / np.abs(Jr).max()
    print("%s %s: max|dW_i|/max|W_i| = %.2e, max|dJ_i|/max|J_i| = %.2e" % (mode, variant, dw, dj),
          flush=True)
    assert dw <= 1e-9 and dj <= 1e-9
    _sum_rule(out)


def test_atom_virial_precision_form():
    s = synth.mof_like(3000, seed=31)
    n = s["pos"].shape[0]
    vel = np.random.default_rng(10).normal(scale=0.01, size=(n, 3))
    ref = R.d3(s["pos"], s["types"], s["cell"], s["pbc"], TAB)
    out = _run(s, "prec", vel)
    dw = np.abs(out["atom_virial"] - ref["atom_virial"]).max()
    print("prec max|dW_i| = %.2e eV (max|W_i| %.2e)" % (dw, np.abs(ref["atom_virial"]).max()),
          flush=True)
    assert dw <= 1e-5
    _sum_rule(out)


def test_atom_virial_surrogate_form():
    """The surrogate pass has its own per-atom variant: the other outputs
    are unchanged by it and the per-atom virials sum to its virial."""
    from paper_2310_05279_amd import d3
    s = synth.mof_like(3000, seed=31)
    n = s["pos"].shape[0]
    vel = np.random.default_rng(11).normal(scale=0.01, size=(n, 3))

    def prep(calc):
        d3.d3_c6_surrogate_init(calc.ctx, 5)
        d3.d3_c6_surrogate_train(calc.ctx, n_samples=60_000, epochs=5, lr=5e-3, lr_final=1e-4,
                                 seed=4, cn_hi=7.0)

    out = _run(s, "surrogate", vel, prep)
    _sum_rule(out)
    J = np.einsum("iab,ib->ia", out["atom_virial"], vel)
    assert np.abs(out["heat_current"] - J).max() <= 1e-12 * np.abs(J).max()


def test_atom_virial_accumulate_and_errors():
    import torch
    from paper_2310_05279_amd import d3
    s = synth.mof_like(800, seed=12)
    n = s["pos"].shape[0]
    calc = d3.D3(TAB)
    calc.build(s["pos"], s["types"], s["cell"], s["pbc"])
    vel = torch.as_tensor(np.random.default_rng(1).normal(size=(n, 3)), device="cuda")
    a = calc.compute(atom_virial=True, velocities=vel)
    b = calc.compute(atom_virial=True, velocities=vel)
    calc.compute(flags=d3.D3_ACCUMULATE, out=b, velocities=vel)
    torch.cuda.synchronize()
    for k in ("atom_virial", "heat_current", "forces", "virial"):
        assert torch.allclose(b[k], 2 * a[k], rtol=1e-14, atol=0), k
    e = torch.zeros(1, dtype=torch.float64, device="cuda")
    hc = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(d3.D3Error) as err:
        d3.d3_evaluate(calc.ctx, calc.pos, e, heat_current=hc)
    assert err.value.code == d3.D3_ERR_INVALID_ARG
    calc.close()


def test_atom_virial_full_size_sampled():
    """The 10^6-atom MOF-like cell: sampled atoms' per-atom virials against
    the oracle's per-atom neighbourhood evaluation."""
    s = synth.mof_like(1_000_000)
    n = s["pos"].shape[0]
    vel = np.random.default_rng(13).normal(scale=0.01, size=(n, 3))
    out = _run(s, "plain", vel)
    idx = np.random.default_rng(14).choice(n, 8, replace=False)
    ref = O.sampled(s["pos"], s["types"], s["cell"], s["pbc"], TAB, idx)
    dw = np.abs(out["atom_virial"][idx] - ref["atom_virial"]).max()
    print("mof1M sampled max|dW_i| = %.2e eV" % dw, flush=True)
    assert dw <= 1e-9 * np.abs(ref["atom_virial"]).max()
    _sum_rule(out)
