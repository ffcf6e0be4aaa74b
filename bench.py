"""Throughput of the D3(BJ) path on one MI355X.

One step = one pass of the whole path on one batch of input: neighbour
build (binning, counting sort, both lists), coordination numbers and
Gaussian weights, the dispersion pass, the chain pass and the FP64
reductions, i.e. energy, forces and virial of the cell.  The headline
workload is the 10^6-atom MOF-like cell (H,C,N,O,Zn 4:6:1:2:1 at 0.04
atoms/A^3, R_pot = 12 A, R_cn = 6 A), the largest single-GPU configuration,
in the plain FP64 form, with the neighbour build in every step; inputs are
resident in HBM before timing starts.  The roofline object is the
dispersion pass's (k_pair) against the FP64 vector peak, with the
algorithmic flops of every unique pair within R_pot; a second entry puts
the list kernel (k_list) against the HBM peak.  The CPU baseline is the C
oracle's cell-list mode on the same cell (all host cores; a single-thread
sample beside it).  Extra fields report the precision and surrogate forms,
Eq. 3 as printed, the 24 000- and 200 000-atom cells, the 500 000-atom
bilayer, long cutoffs and velocity-Verlet NVE.

Prints ONE JSON line.  Usage: python bench.py [--steps K] [--warmup W]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("D3 atom-steps/s (E+F+virial), surrogate/FP32 vs plain at "
          "≤1e-4 eV/Å force")
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0


# the D3 variants the paper sets aside, as options of the headline step
_ZERO = dict(damping="zero", s6=1.0, s8=0.722, rs6=1.217, rs8=1.0)
VARIANTS = {"bj": {}, "zero": _ZERO, "bj_atm": dict(s9=1.0, r_atm=6.0),
            "zero_atm": dict(_ZERO, s9=1.0, r_atm=6.0)}

# HBM bytes per launch of the dispersion pass on the 10^6-atom cell, from two
# rocprofv3 --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch), each scaled by what the same counter read for a 512 MiB device
# copy.  The figure belongs to the kernel sources it was taken with: when
# their hash differs it is not used (None: not measured on these sources).
PAIR_TRAFFIC = {
    "fetch_kib": 2074469.1, "write_kib": 70794.4,
    "fetch_scale": 524288.0 / 262157.1, "write_scale": 524288.0 / 524288.0,
    "sources": ("disp.hip", "d3_device.h", "d3_internal.h"),
    "sha256": "12cd1357c66cc4fb72d6e32d9907e78d",
}


def _sources_hash(names):
    import hashlib
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2310_05279_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:32]


def pair_traffic_bytes(t=None):
    t = PAIR_TRAFFIC if t is None else t
    if t is None or _sources_hash(t["sources"]) != t["sha256"]:
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def _flops_per_pair(ki, kj):
    """Algorithmic FP64 operations of one unique dispersion pair within
    R_pot (energy, both forces, virial and both dE/dn terms): 56 for the
    distance, damping, force and virial arithmetic, 4 K_i K_j for the
    bilinear form C6 = w_i^T M w_j with its two CN derivatives, and
    2 K_i + 4 K_j for the weight terms of the atom that evaluates the pair
    and of its partner, averaged over the two ends of the unordered pair:
    56 + 4 K_i K_j + 3 (K_i + K_j).  Divisions count as one."""
    return 56.0 + 4.0 * ki * kj + 3.0 * (ki + kj)


def unique_pair_counts(system, r_pot):
    """Unique pairs (i < j, images included) within r_pot per element pair
    (e <= f) of a cubic periodic cell: {(e, f): count}.  Input statistics
    only (k-d trees over the wrapped positions)."""
    from scipy.spatial import cKDTree
    box = system["cell"][0, 0]
    assert np.allclose(system["cell"], np.eye(3) * box) and np.all(system["pbc"])
    pos = np.mod(system["pos"], box)
    types = np.asarray(system["types"])
    els = np.unique(types)
    trees = {e: cKDTree(pos[types == e], boxsize=box) for e in els}
    out = {}
    for a, e in enumerate(els):
        for f in els[a:]:
            c = int(trees[e].count_neighbors(trees[f], r_pot))
            if e == f:
                c = (c - trees[e].n) // 2
            out[(int(e), int(f))] = c
    return out


def algorithmic_pair_flops(system, table, r_pot):
    """Sum of _flops_per_pair over the unique pairs within r_pot, and the
    number of those pairs."""
    k = np.asarray(table["n_ref"], dtype=np.float64)
    counts = unique_pair_counts(system, r_pot)
    flops = sum(c * _flops_per_pair(k[e], k[f]) for (e, f), c in counts.items())
    return float(flops), int(sum(counts.values()))


class Runner:
    def __init__(self, system, table, mode="plain", skin=0.0, per_atom=False, **prm):
        import torch
        from paper_2310_05279_amd import d3
        self.torch, self.d3 = torch, d3
        self.dev = torch.device("cuda", 0)
        self.calc = d3.D3(table, mode=mode, skin=skin, **prm)
        self.calc.build(system["pos"], system["types"], system["cell"], system["pbc"])
        self.n = self.calc.n
        self.out = {"energy": torch.zeros(1, dtype=torch.float64, device=self.dev),
                    "forces": torch.zeros((self.n, 3), dtype=torch.float64, device=self.dev),
                    "virial": torch.zeros((3, 3), dtype=torch.float64, device=self.dev),
                    "atom_energy": None}
        # per-atom virials (Eq. 7) and heat currents (Eq. 8) at 300 K-like velocities
        self.per_atom = per_atom
        if per_atom:
            self.out["atom_virial"] = torch.zeros((self.n, 3, 3), dtype=torch.float64,
                                                  device=self.dev)
            self.out["heat_current"] = torch.zeros((self.n, 3), dtype=torch.float64,
                                                   device=self.dev)
            rng = np.random.default_rng(300)
            self.vel = torch.as_tensor(rng.normal(scale=0.01, size=(self.n, 3)), device=self.dev)
        self.stream = torch.cuda.current_stream()

    def step(self, rebuild=True):
        """One step: with rebuild, the neighbour build from the positions
        (D3_REBUILD, as for a new configuration), then the evaluation."""
        d3, c = self.d3, self.calc
        fl = d3.D3_REBUILD if rebuild else 0
        if self.per_atom:
            o = self.out
            d3.d3_evaluate(c.ctx, c.pos, o["energy"], o["forces"], o["virial"], None,
                           o["atom_virial"], self.vel, o["heat_current"], fl, self.stream)
        else:
            d3.d3_energy_forces_virial(c.ctx, c.pos, self.out["energy"], self.out["forces"],
                                       self.out["virial"], None, fl, self.stream)

    def timed(self, steps, warmup, rebuild=True, phases=False):
        """Mean ms per step over `steps` steps after `warmup` untimed ones.
        With phases, the library also records HIP events around each pass
        of these same steps (on its stream; the events are created during
        the warm-up) and the per-pass means are returned as well."""
        torch, d3 = self.torch, self.d3
        if phases:
            d3.d3_set_timing(self.calc.ctx, 1)
        for _ in range(warmup):
            self.step(rebuild)
        torch.cuda.synchronize()
        self.calc.status()
        if phases:
            d3.d3_set_timing(self.calc.ctx, 1)  # drops the warm-up's events
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(self.stream)
        for _ in range(steps):
            self.step(rebuild)
        t1.record(self.stream)
        torch.cuda.synchronize()
        self.calc.status()
        ms = t0.elapsed_time(t1) / steps
        if not phases:
            return ms
        t = d3.d3_get_timing(self.calc.ctx)
        d3.d3_set_timing(self.calc.ctx, 0)
        ph = {k: (v / calls if calls else 0.0) for k, (v, calls) in t.items()}
        ph["build"] = ph["sort"] + ph["list"]
        return ms, ph

    def graphed(self, steps, warmup, rebuild=True):
        """Time `steps` replays of a HIP graph holding one whole step (the
        same library calls as step(), captured once on a side stream).  The
        kernels are the eager ones; a graph only removes the launch gaps."""
        torch = self.torch
        s = torch.cuda.Stream()
        eager_stream = self.stream
        self.stream = s
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            for _ in range(max(warmup, 2)):
                self.step(rebuild)
        torch.cuda.synchronize()
        self.calc.status()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            self.step(rebuild)
        torch.cuda.synchronize()
        # replay() launches on torch's current stream: the events go there
        cur = torch.cuda.current_stream()
        for _ in range(warmup):
            g.replay()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(cur)
        for _ in range(steps):
            g.replay()
        t1.record(cur)
        torch.cuda.synchronize()
        self.calc.status()
        self.stream = eager_stream
        del g
        return t0.elapsed_time(t1) / steps

    def phases(self, steps, rebuild=True):
        d3 = self.d3
        d3.d3_set_timing(self.calc.ctx, 1)
        for _ in range(steps):
            self.step(rebuild)
        self.torch.cuda.synchronize()
        t = d3.d3_get_timing(self.calc.ctx)
        d3.d3_set_timing(self.calc.ctx, 0)
        ph = {k: (ms / calls if calls else 0.0) for k, (ms, calls) in t.items()}
        ph["build"] = ph["sort"] + ph["list"]
        return ph

    def close(self):
        self.calc.close()


def cpu_model():
    """The host CPU's model name from /proc/cpuinfo (None if unreadable)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(system, table, n_threads=0, n_eval=None):
    """The C FP64 oracle's cell-list mode timed on the host for one E+F+W
    evaluation of the cell (n_eval: the passes of that many atoms only, a
    timing sample).  Returns the result, the seconds and the threads."""
    from oracle import d3_ref
    t0 = time.perf_counter()
    ref = d3_ref.d3(system["pos"], system["types"], system["cell"], system["pbc"], table,
                    cells=True, n_threads=n_threads, n_eval=n_eval)
    dt = time.perf_counter() - t0
    return ref, dt, d3_ref.threads(n_threads)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the precision/surrogate/other-cell/MD fields")
    ap.add_argument("--no-flops", action="store_true",
                    help="skip the unique-pair count (roofline fields become null)")
    ap.add_argument("--sur-epochs", type=int, default=3000)
    ap.add_argument("--md-steps", type=int, default=200)
    ap.add_argument("--graph", action="store_true",
                    help="also time the headline step replayed from a HIP graph")
    ap.add_argument("--variant", choices=sorted(VARIANTS), default="bj",
                    help="the headline step with zero damping and/or the three-body term "
                         "(for profiling those passes; no roofline or CPU baseline then)")
    ap.add_argument("--form", choices=("plain", "prec", "sur"), default="plain",
                    help="the headline step in the precision form, or with the surrogate C6 "
                         "trained for --sur-epochs epochs first (for profiling their passes; "
                         "no roofline or CPU baseline then)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run 3 plain device-to-device copies of this many MiB "
                         "(a known-size reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the D3 path here is single-GPU "
              "(it is not sharded across GPUs); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    table = synth.make_table()
    system = synth.mof_like(1_000_000)
    n = system["pos"].shape[0]
    log("workload mof_1M plain %s: warmup %d, steps %d" % (args.variant, args.warmup, args.steps))
    headline_kw = VARIANTS[args.variant]
    if args.variant != "bj" or args.form != "plain":
        args.no_flops = args.no_cpu_baseline = True

    run = Runner(system, table, "surrogate" if args.form == "sur" else args.form, **headline_kw)
    if args.form == "sur":
        # the surrogate trained on this cell's CN box (99.9th percentile + 0.5)
        from paper_2310_05279_amd import d3 as d3mod
        cn = run.calc.coordination().cpu().numpy()
        cn_hi = float(np.percentile(cn, 99.9) + 0.5)
        d3mod.d3_c6_surrogate_init(run.calc.ctx, 5)
        d3mod.d3_c6_surrogate_train(run.calc.ctx, n_samples=1_000_000, epochs=args.sur_epochs,
                                    lr=1e-2, lr_final=1e-6, seed=4, cn_hi=cn_hi)
        log("surrogate trained for %d epochs on [0, %.3f]^2" % (args.sur_epochs, cn_hi))
    ms = run.timed(args.steps, args.warmup)
    value = n / (ms * 1e-3)
    ms_graph = run.graphed(args.steps, args.warmup) if args.graph else None
    # the same K steps again with HIP events around each pass (the events add
    # about 1 % to a step, so the headline value comes from the clean region)
    ms_ev, ph = run.timed(args.steps, 2, phases=True)
    stats = run.calc.stats()
    ms_eval = run.timed(args.steps, 3, rebuild=False)
    res_f = run.out["forces"].cpu().numpy()
    res_e = float(run.out["energy"].item())
    res_w = run.out["virial"].cpu().numpy()
    run.close()
    log("plain %.4f ms/step, eval only %.4f, phases %s" % (ms, ms_eval, ph))

    roofline = None
    if not args.no_flops:
        log("counting unique pairs within R_pot per element pair")
        flops, npairs = algorithmic_pair_flops(system, table, 12.0)
        pair_ms = ph["pair"]
        achieved = flops / (pair_ms * 1e-3) / 1e12
        roofline = {"kernel": "k_pair<fp64> (dispersion pass)", "bound": "alu",
                    "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": pair_traffic_bytes(),
                    "algorithmic_flops_per_launch": flops, "unique_pairs": npairs,
                    "flops_per_unique_pair": flops / npairs, "avg_kernel_ms": pair_ms,
                    "kernel_ms_source": "HIP events around the pass on the library's stream, "
                                        "mean over %d timed steps" % args.steps}
        if roofline["traffic"] is not None:
            gbs = roofline["traffic"] / (pair_ms * 1e-3) / 1e9
            roofline["hbm_GBs"] = gbs
            roofline["hbm_frac"] = gbs / HBM_PEAK_GBS
        # the list kernel against HBM: it must read every sorted position
        # (32 B) and write both lists (4 B per entry) and both counts
        entries = stats["mean_pot"] * n + stats["mean_cn"] * n
        list_bytes = 40.0 * n + 4.0 * entries
        list_gbs = list_bytes / (ph["list"] * 1e-3) / 1e9
        roofline["other"] = [{"kernel": "k_list (neighbour lists)", "bound": "hbm",
                              "achieved": list_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": list_gbs / HBM_PEAK_GBS,
                              "algorithmic_bytes_per_launch": list_bytes,
                              "avg_kernel_ms": ph["list"]}]

    extra = {"ms_per_step_with_phase_events": ms_ev,
             "ms_per_step_eval_only": ms_eval,
             "atom_steps_per_s_eval_only": n / (ms_eval * 1e-3),
             "ms_per_step_graph_replay": ms_graph,
             "phase_ms": ph, "list_stats": stats}

    cpu = None
    if not args.no_cpu_baseline:
        log("CPU baseline: cell-list oracle, all threads, 10^6 atoms")
        ref, dt, threads = cpu_baseline(system, table)
        extra["plain_vs_oracle"] = {
            "abs_dE_per_atom": abs(res_e - ref["energy"]) / n,
            "max_abs_dF": float(np.abs(res_f - ref["forces"]).max()),
            "max_abs_dW": float(np.abs(res_w - ref["virial"]).max()),
            "max_abs_W": float(np.abs(ref["virial"]).max())}
        del ref
        m1 = 250_000
        log("CPU baseline: one thread, passes of %d atoms" % m1)
        _, dt1, _ = cpu_baseline(system, table, n_threads=1, n_eval=m1)
        cpu = {"value": n / dt, "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
               "sample": "one full FP64 E+F+W evaluation of the same 10^6-atom cell by the C "
                         "oracle's cell-list mode on %d OpenMP threads (%.1f s)" % (threads, dt),
               "cpu_model": cpu_model(), "host_threads": len(os.sched_getaffinity(0)),
               "single_thread": {"value": m1 / dt1, "unit": "atom-steps/s", "cores": 1,
                                 "sample": "the CN, dispersion and chain passes of %d of the "
                                           "cell's atoms, one thread (%.1f s)" % (m1, dt1)}}
        log("CPU baseline %s" % json.dumps(cpu))

    if not args.no_extra:
        from paper_2310_05279_amd import d3 as d3mod

        def forms(big, steps, modes, weights=None):
            """Speed of each form on a cell, and the deviation of the other
            forms from the plain FP64 result."""
            entry, ref = {}, None
            nbig = big["pos"].shape[0]
            for mode in modes:
                run = Runner(big, table, mode)
                if mode == "surrogate":
                    d3mod.d3_c6_surrogate_set_weights(run.calc.ctx, weights)
                msb = run.timed(steps, 2)
                phb = run.phases(5)
                got = (run.out["forces"].cpu().numpy(), float(run.out["energy"].item()),
                       run.out["virial"].cpu().numpy())
                run.close()
                entry[mode] = {"atom_steps_per_s": nbig / (msb * 1e-3),
                               "ms_per_step": msb, "phase_ms": phb}
                if mode == "plain":
                    ref = got
                elif ref is not None:
                    entry[mode].update({
                        "max_abs_dF_vs_plain": float(np.abs(got[0] - ref[0]).max()),
                        "abs_dE_per_atom_vs_plain": abs(got[1] - ref[1]) / nbig,
                        "max_abs_dW_vs_plain": float(np.abs(got[2] - ref[2]).max())})
            if "literal" in entry and "surrogate" in entry:
                entry["surrogate"]["speed_vs_literal_eq3"] = (entry["literal"]["ms_per_step"] /
                                                             entry["surrogate"]["ms_per_step"])
            return entry

        # the precision form on the headline cell, with its pair pass against
        # the FP32 peak on the same flop count
        run = Runner(system, table, "prec")
        ms_p = run.timed(args.steps, args.warmup)
        php = run.phases(max(10, args.steps // 2))
        fp = run.out["forces"].cpu().numpy()
        ep = float(run.out["energy"].item())
        wp = run.out["virial"].cpu().numpy()
        run.close()
        extra["prec_f32"] = {"atom_steps_per_s": n / (ms_p * 1e-3), "ms_per_step": ms_p,
                             "phase_ms": php, "pair_time_vs_plain": php["pair"] / ph["pair"],
                             "max_abs_dF_vs_plain": float(np.abs(fp - res_f).max()),
                             "abs_dE_per_atom_vs_plain": abs(ep - res_e) / n,
                             "max_abs_dW_vs_plain": float(np.abs(wp - res_w).max())}
        if roofline is not None:
            a32 = roofline["algorithmic_flops_per_launch"] / (php["pair"] * 1e-3) / 1e12
            extra["prec_f32"]["pair_roofline"] = {"achieved_TFLOPs": a32,
                                                  "peak_TFLOPs": FP32_VECTOR_PEAK_TFLOPS,
                                                  "frac": a32 / FP32_VECTOR_PEAK_TFLOPS}
        log("prec %s" % json.dumps(extra["prec_f32"]))

        # 24 000-atom cell: plain, per-atom virial, the surrogate (trained here
        # on 10^6 exact-labelled CN pairs over [0, 99.9th CN percentile + 0.5]^2)
        # and Eq. 3 as printed
        small = synth.mof_like(24000)
        ns = small["pos"].shape[0]
        run = Runner(small, table, "plain", per_atom=True)
        ms_a = run.timed(args.steps * 5, args.warmup)
        run.close()
        run = Runner(small, table, "surrogate")
        cn = run.calc.coordination().cpu().numpy()
        cn_hi = float(np.percentile(cn, 99.9) + 0.5)
        d3mod.d3_c6_surrogate_init(run.calc.ctx, 5)
        t0 = time.perf_counter()
        loss = d3mod.d3_c6_surrogate_train(run.calc.ctx, n_samples=1_000_000,
                                           epochs=args.sur_epochs, lr=1e-2, lr_final=1e-6,
                                           seed=4, cn_hi=cn_hi)
        t_train = time.perf_counter() - t0
        weights = d3mod.d3_c6_surrogate_get_weights(run.calc.ctx)
        run.close()
        e24 = forms(small, args.steps * 5, ("plain", "prec", "literal", "surrogate"), weights)
        e24["plain_with_atom_virial"] = {"atom_steps_per_s": ns / (ms_a * 1e-3),
                                         "ms_per_step": ms_a}
        e24["surrogate"].update({"train_s": t_train, "train_loss": loss, "cn_hi": cn_hi})
        extra["mof_24000"] = e24
        log("mof_24000 %s" % json.dumps(e24))

        for name, big, steps, modes in (
                ("mof_200k", synth.mof_like(200_000), 10,
                 ("plain", "prec", "literal", "surrogate")),
                ("graphene_500k", synth.bilayer_graphene(250, 500, seed=500000), 10,
                 ("plain", "prec"))):
            extra[name] = forms(big, steps, modes, weights)
            log("%s %s" % (name, json.dumps(extra[name])))

        # the variants the paper sets aside: zero damping, the three-body term
        # (r_atm = R_cn = 6 A) and both, on the headline cell, plain FP64
        variants = {}
        for vname, kw in (("zero_damping", VARIANTS["zero"]), ("bj_atm", VARIANTS["bj_atm"]),
                          ("zero_atm", VARIANTS["zero_atm"])):
            run = Runner(system, table, "plain", **kw)
            msv = run.timed(10, 2)
            phv = run.phases(5)
            run.close()
            variants[vname] = {"atom_steps_per_s": n / (msv * 1e-3), "ms_per_step": msv,
                               "phase_ms": phv}
        extra["variants_mof_1M"] = variants
        log("variants %s" % json.dumps(variants))

        # long cutoffs on the 24 000-atom cell, R_cn = R_pot / 2: speed, and the
        # force error of each cutoff against the 50 A result (plain FP64)
        sweep, f50 = {}, None
        for rp in (50.0, 40.0, 30.0, 20.0, 12.0):
            run = Runner(small, table, "plain", r_pot=rp, r_cn=rp / 2)
            msc = run.timed(10, 2)
            phc = run.phases(5)
            fc = run.out["forces"].cpu().numpy()
            st = run.calc.stats()
            run.close()
            if f50 is None:
                f50 = fc
            sweep["%g" % rp] = {"r_cn": rp / 2, "atom_steps_per_s": ns / (msc * 1e-3),
                                "ms_per_step": msc, "phase_ms": phc,
                                "mean_entries_pot": st["mean_pot"],
                                "force_rmse_vs_50A": float(np.sqrt(((fc - f50) ** 2).mean())),
                                "force_maxerr_vs_50A": float(np.abs(fc - f50).max())}
        extra["cutoff_sweep_mof24000"] = sweep
        log("cutoff sweep %s" % json.dumps(sweep))

        # velocity-Verlet NVE on the 10^6-atom cell: 300 K Maxwell start, 1 fs,
        # lists with a 1 A skin rebuilt when an atom moved more than 0.5 A
        vel0, mass = synth.maxwell_velocities(system["types"], 300.0, seed=300)
        md = {}
        for mode in ("plain", "prec", "surrogate"):
            run = Runner(system, table, mode, skin=1.0)
            if mode == "surrogate":
                d3mod.d3_c6_surrogate_set_weights(run.calc.ctx, weights)
            pos = run.calc.pos.clone()
            vel = torch.as_tensor(vel0, device="cuda")
            mss = torch.as_tensor(mass, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            thermo, reb = d3mod.d3_md_nve(run.calc.ctx, args.md_steps, 1.0, pos, vel, mss,
                                          every=args.md_steps)
            dt = time.perf_counter() - t0
            run.close()
            md[mode] = {"atom_steps_per_s": n * args.md_steps / dt,
                        "ms_per_step": 1e3 * dt / args.md_steps, "rebuilds": reb,
                        "etot_drift_per_atom_eV": float((thermo[-1, 2] - thermo[0, 2]) / n)}
        extra["md_nve_mof_1M"] = md
        log("md %s" % json.dumps(md))

        # the paper's own throughput shape (Table I): a 40 000-atom AB bilayer
        # (100 x 100 supercell), one step with a build, and NVE MD as above
        bl = synth.bilayer_graphene(100, 100, seed=40000)
        nbl = bl["pos"].shape[0]
        vb, mb = synth.maxwell_velocities(bl["types"], 300.0, seed=301)
        entry = {"n_atoms": nbl}
        for mode in ("plain", "prec"):
            run = Runner(bl, table, mode)
            msb = run.timed(50, 5)
            run.close()
            run = Runner(bl, table, mode, skin=1.0)
            pos = run.calc.pos.clone()
            vel = torch.as_tensor(vb, device="cuda")
            mss = torch.as_tensor(mb, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            thermo, reb = d3mod.d3_md_nve(run.calc.ctx, args.md_steps, 1.0, pos, vel, mss,
                                          every=args.md_steps)
            dt = time.perf_counter() - t0
            run.close()
            entry[mode] = {"atom_steps_per_s_build_every_step": nbl / (msb * 1e-3),
                           "ms_per_step_build_every_step": msb,
                           "md_atom_steps_per_s": nbl * args.md_steps / dt,
                           "md_ms_per_step": 1e3 * dt / args.md_steps, "md_rebuilds": reb,
                           "md_etot_drift_per_atom_eV":
                               float((thermo[-1, 2] - thermo[0, 2]) / nbl)}
        extra["bilayer_40k"] = entry
        log("bilayer 40k %s" % json.dumps(entry))

    line = {"metric": METRIC, "value": value, "unit": "atom-steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": {"plain": "f64", "prec": "f32 (pair arithmetic; f64 sums)",
                      "sur": "bf16 MFMA + f32 (surrogate C6); f64 pair terms"}[args.form],
            "data": "synthetic",
            "config": {"workload": "mof_like_1M (10^6 atoms, H,C,N,O,Zn 4:6:1:2:1, 0.04 "
                                   "atoms/A^3, seed 1000000; synthetic D3 table seed 2310; "
                                   "R_pot 12 A, R_cn 6 A; plain FP64; E+F+virial with the "
                                   "neighbour build in every step)" +
                                   ("" if args.variant == "bj" else
                                    "; variant %s" % args.variant) +
                                   {"plain": "", "prec": "; precision form",
                                    "sur": "; surrogate C6 form (%d training epochs)"
                                           % args.sur_epochs}[args.form],
                       "n_atoms": n, "parallelism": "single GPU"},
            "roofline": roofline, "cpu_baseline": cpu, "extra": extra}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
