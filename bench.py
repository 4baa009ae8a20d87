"""Throughput benchmark of the energy+force path on one MI355X.

Default workload: the ragged batch of 512 independent non-periodic solutes
(10-120 atoms, H/C/N/O/S/F/Cl), evaluated in one call per step with the
dense layers in bfloat16 (float32 accumulate).  Beside it the same batch is
run the plain way: float32 dense layers, one system per call, sequentially
on one stream.  One atom-eval = energy + forces of one atom.

Prints one JSON line: the metric, its value and unit, the timed steps, the
per-stage times, the dominant kernel's roofline and the oracle's CPU
baseline.
"""
from __future__ import annotations

import argparse
import contextlib
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VALU_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--workload", default="ragged512",
                   choices=["ragged512", "water2001", "protein100k", "cluster24", "serve", "copy",
                            "hybrid", "snapshots"])
    p.add_argument("--precision", default="bf16", choices=["bf16", "fp32"])
    p.add_argument("--model", default="ani", choices=["ani", "dp"],
                   help="descriptor family: ANI AEV (default) or DeepPot-style local frame")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--plain-passes", type=int, default=2)
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--quiet", action="store_true")
    p.add_argument("--requests", type=int, default=4000, help="serving: requests in the trace")
    p.add_argument("--rate", type=float, default=2000.0, help="serving: Poisson arrival rate (1/s)")
    p.add_argument("--req-steps", type=int, default=50, help="serving: steps per request")
    p.add_argument("--plain-requests", type=int, default=48, help="serving: sample for the plain path")
    p.add_argument("--graphs", default="both", choices=["on", "off", "both"],
                   help="serving: iterations replayed from recorded graphs, launched directly, or both")
    return p.parse_args()


@contextlib.contextmanager
def no_gc_pauses():
    """A timed region without Python garbage-collection pauses: a full
    collection over the interpreter's objects (torch alone holds hundreds of
    thousands) takes tens of milliseconds on the host and would be charged
    to whatever step it interrupts.  Collect first, keep the collector off
    until the region ends."""
    gc.collect()
    gc.disable()
    try:
        yield
    finally:
        gc.enable()


def cpu_model() -> str:
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def say(args, *a):
    if not args.quiet:
        print("[bench]", *a, file=sys.stderr, flush=True)


def workload(name, kind="ani"):
    import synth
    if kind == "dp":
        mk, tag = synth.make_dp_model, "; DeepPot-style local-frame descriptor (rc 6 A, 120 slots, 480 features)"
    else:
        mk, tag = synth.make_model, ""
    if name == "ragged512":
        return synth.config2(), mk(0), "ragged batch: 512 non-periodic solutes, 10-120 atoms" + tag
    if name == "water2001":
        return synth.make_batch([synth.config1()]), mk(0), "periodic water box, 2001 atoms, L=27.1 A" + tag
    if name == "protein100k":
        return (synth.make_batch([synth.config3()]), mk(3, n_ensemble=8),
                "periodic solvated-protein-like box, 100,002 atoms, L=101 A, ensemble of 8 networks" + tag)
    return synth.make_batch([synth.config0()]), mk(0), "24-atom cluster" + tag


def dp_counts(model, batch, c, s):
    """Work of the DeepPot-style descriptor kernels, from the library's own
    neighbour lists (distances recomputed here in float64): valid entries
    (inside rc), same-species comparisons of the in-bucket ranking
    (sum over centres and species of n_s^2), kept slots, centres."""
    cnt, ent = model.neighbors(c, s, batch.boxes, batch.offsets, capacity=model_cap(model))
    cnt = cnt.cpu().numpy()
    ent = ent.cpu().numpy()
    sys_of = np.repeat(np.arange(batch.n_systems), np.diff(batch.offsets))
    x = batch.coords.astype(np.float64)
    rc, sel = model.spec.aev["rc"], np.asarray(model.spec.aev["sel"])
    entries = comps = kept = 0
    for i in range(batch.n_atoms):
        e = ent[i, :min(cnt[i], ent.shape[1])]
        if len(e) == 0:
            continue
        L = batch.boxes[sys_of[i]].astype(np.float64)
        d = x[e[:, 0]] + e[:, 1:4] * L - x[i]
        inside = (d * d).sum(1) < rc * rc
        ns = np.bincount(batch.species[e[inside, 0]], minlength=len(sel))
        entries += int(inside.sum())
        comps += int((ns.astype(np.int64) ** 2).sum())
        kept += int(np.minimum(ns, sel).sum())
    return entries, comps, kept, batch.n_atoms


def pair_triplet_counts(model, batch, c, s):
    """Radial pairs and angular triplets of the batch, from the library's own
    neighbour lists (distances recomputed here in float64)."""
    cnt, ent = model.neighbors(c, s, batch.boxes, batch.offsets, capacity=model_cap(model))
    cnt = cnt.cpu().numpy()
    ent = ent.cpu().numpy()
    sys_of = np.repeat(np.arange(batch.n_systems), np.diff(batch.offsets))
    x = batch.coords.astype(np.float64)
    rc_r, rc_a = model.spec.aev["rc_rad"], model.spec.aev["rc_ang"]
    n_pairs = 0
    n_trip = 0
    for i in range(batch.n_atoms):
        e = ent[i, :min(cnt[i], ent.shape[1])]
        if len(e) == 0:
            continue
        L = batch.boxes[sys_of[i]].astype(np.float64)
        d = x[e[:, 0]] + e[:, 1:4] * L - x[i]
        r = np.sqrt((d * d).sum(1))
        n_pairs += int((r < rc_r).sum())
        na = int((r < rc_a).sum())
        n_trip += na * (na - 1) // 2
    return n_pairs, n_trip


PROBE_STEPS = 5


def probe_stages(model, call):
    """Mean stage times of PROBE_STEPS calls with every stage boundary
    recorded (untimed steps)."""
    import torch
    model.set_timing(True)
    for _ in range(PROBE_STEPS):
        call()
    torch.cuda.synchronize()
    stages = model.stage_timings()
    model.set_timing(False)
    return stages


def size_capacity(model, batch, c, sp, N, S):
    """Neighbour capacity = largest neighbour count, rounded up (LDS use of
    the AEV kernels scales with it)."""
    model.reserve(N, S, 1024)
    model.energy_forces(c, sp, batch.boxes, batch.offsets, forces=False)
    mx = model.status()
    cap = min(1024, (mx + 8 + 31) // 32 * 32)
    model.reserve(N, S, cap)
    model._bench_cap = cap
    return cap


def model_cap(model):
    return getattr(model, "_bench_cap", 256)


def model_cutoff(spec):
    """Neighbour cutoff of a model (the larger descriptor cutoff)."""
    a = spec.aev if isinstance(spec.aev, dict) else vars(spec.aev)
    return max(float(a.get(k, 0.0)) for k in ("rc_rad", "rc_ang", "rc"))


def cell_count(batch, rc):
    """Cells of the library's grid for a call on this batch: per periodic
    system floor(L / rc) per axis (at least 1, at most 1,024), a quarter of
    the atom count for a non-periodic bounding-box grid."""
    total = 0
    for k in range(batch.n_systems):
        n = int(batch.offsets[k + 1] - batch.offsets[k])
        b = np.asarray(batch.boxes[k], np.float64)
        if np.all(b > 0):
            nc = [min(1024, max(1, int(np.floor(x / (rc * (1 + 1e-5)))))) for x in b]
            total += nc[0] * nc[1] * nc[2]
        else:
            total += max(1, n // 4)
    return total


# Algorithmic work of the AEV stages, counted from the formulas (flops of the
# float32 vector unit; a transcendental (exp, log, sin/cos, sqrt, reciprocal)
# counts 4, its issue cost relative to an add or multiply):
#   radial pair:  per shift  (R - Rs), square, * eta, exp, * fc, accumulate
#                 = 5 + 4 = 9; x16 shifts = 144; + distance (8 + sqrt 4) and
#                 cutoff (2 + cos 4) = 18                      -> 162
#   triplet:      geometry (dot 5, cross 9 + sqrt, 1/(RjRk), cos/sin 2) = 25;
#                 per angle shift: cos(theta - theta_s) 3, 1 + c 1, log 4,
#                 * zeta + const 2, exp2 4 = 14, x8 = 112;
#                 per radial shift: Rbar - Rs, square, * eta, exp 4 = 7, x4 = 28;
#                 fc_j fc_k 1; per (a, r) product and accumulate 2, x32 = 64
#                                                               -> 230
# The backward pass differentiates the same terms: radial 2x (dE/dR of each
# shift's Gaussian and cutoff), triplet ~2.2x (derivatives through cos, sin,
# R_j, R_k and the cutoff product), i.e. 324 and 510.
FLOP_RADIAL_FWD = 162
FLOP_TRIPLET_FWD = 230
FLOP_RADIAL_BWD = 324
FLOP_TRIPLET_BWD = 510

# DeepPot-style descriptor, counted the same way (float64 operations count 2,
# their issue cost on the float32 vector unit):
#   forward:  per valid entry the float64 order key (3 subtractions, 3 image
#             products, 3 additions, 3 squares, 2 additions: 14 -> 28);
#             per same-species comparison of the ranking 1;
#             per kept slot |d| (5 + sqrt 4), 1/R 4, three projections 15 -> 28;
#             per centre the frame (normalise 2 vectors, Gram-Schmidt, cross
#             product) ~ 40
#   backward: per kept slot the vector (9 + 4) again, 1/R 4, three projections
#             15, s 7 + 2, dE/dd 3 x 8, frame sums 18, virial 18, force sums
#             and the neighbour's force 6 -> 107; per centre the frame again
#             (40) and its chain rule (~90) -> 130
FLOP_DP_ENTRY_FWD = 28
FLOP_DP_COMPARE = 1
FLOP_DP_SLOT_FWD = 28
FLOP_DP_CENTRE_FWD = 40
FLOP_DP_SLOT_BWD = 107
FLOP_DP_CENTRE_BWD = 130


def mlp_flops(spec, species):
    """2 * MACs of forward and backward (input gradient) dense layers."""
    per = []
    for w in spec.widths:
        macs = sum(w[l] * w[l + 1] for l in range(len(w) - 1))
        per.append(macs)
    per = np.array(per, dtype=np.float64)
    fwd = 2.0 * per[species].sum() * spec.n_ensemble
    bwd = 2.0 * (per[species] - np.array([w[-2] for w in spec.widths])[species]).sum() * spec.n_ensemble
    return fwd, bwd


# Kernel sources whose hash a counter summary records: the HBM byte counts
# it holds describe the kernel as it was built from exactly these files.
KERNEL_SOURCES = {
    "k_aev_fwd": ["paper_2207_14276_amd/csrc/aev.hip", "paper_2207_14276_amd/csrc/internal.h",
                  "paper_2207_14276_amd/csrc/wave.h"],
    "k_aev_bwd": ["paper_2207_14276_amd/csrc/aev.hip", "paper_2207_14276_amd/csrc/internal.h",
                  "paper_2207_14276_amd/csrc/wave.h", "paper_2207_14276_amd/csrc/fixed.h"],
    "k_aev_bwd_sys": ["paper_2207_14276_amd/csrc/aev.hip", "paper_2207_14276_amd/csrc/internal.h",
                      "paper_2207_14276_amd/csrc/wave.h", "paper_2207_14276_amd/csrc/fixed.h"],
    "k_aev_bwd_cells": ["paper_2207_14276_amd/csrc/aev.hip", "paper_2207_14276_amd/csrc/internal.h",
                        "paper_2207_14276_amd/csrc/wave.h", "paper_2207_14276_amd/csrc/fixed.h"],
    "k_dp_fwd": ["paper_2207_14276_amd/csrc/deeppot.hip", "paper_2207_14276_amd/csrc/internal.h",
                 "paper_2207_14276_amd/csrc/wave.h"],
    "k_dp_bwd": ["paper_2207_14276_amd/csrc/deeppot.hip", "paper_2207_14276_amd/csrc/internal.h",
                 "paper_2207_14276_amd/csrc/wave.h"],
    "k_dp_bwd_sys": ["paper_2207_14276_amd/csrc/deeppot.hip", "paper_2207_14276_amd/csrc/internal.h",
                     "paper_2207_14276_amd/csrc/wave.h"],
    "k_gemm": ["paper_2207_14276_amd/csrc/mlp.hip", "paper_2207_14276_amd/csrc/internal.h"],
}


def kernel_source_hash(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def read_summary(path):
    """`key: value` lines of a counter summary (other lines ignored)."""
    out = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#", "|")):
                k, v = line.split(":", 1)
                out[k.strip()] = v.strip()
    return out


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the
    counter reads for a plain 1 GiB copy); None when there is no summary or
    the kernel's source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_hbm.txt")
    if not os.path.exists(path):
        return None
    d = read_summary(path)
    if d.get("source_sha256") != kernel_source_hash(kernel):
        return None
    return int(float(d["traffic_bytes_per_launch"]))


def copy_probe(args):
    """A plain device-to-device copy of 1 GiB: the known-size reference for
    the HBM byte counters (FETCH_SIZE, WRITE_SIZE) of rocprofv3."""
    import torch
    n = 1 << 28  # float32 elements = 1 GiB
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(max(1, args.steps)):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n,
                      "launches": max(1, args.steps)}), flush=True)


def serve_bench(args):
    """Serving: a Poisson stream of requests (log-uniform 20-5000 atoms, half
    periodic water boxes, half dense solutes), each a random walk of
    `req_steps` steps, through the library's continuous-batching server
    (bfloat16 dense layers, persistent neighbour lists with a 1 A skin,
    memory-bound admission); beside it a seeded sample of the same requests
    through the plain path (float32, one request and one step per call,
    fresh lists)."""
    import torch
    import synth
    from paper_2207_14276_amd import NNPModel
    from paper_2207_14276_amd.serve import Request, Server, replay

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    spec = synth.make_model(0)
    say(args, f"generating {args.requests} requests")
    trace = synth.request_trace(args.requests, seed=4, rate=args.rate, n_steps=args.req_steps)
    sizes = np.array([r.system.n for r in trace])
    cap = 640   # dense 5000-atom solutes: ~550 neighbours within rc + skin
    model = NNPModel(spec, "bf16")
    slots = int(sizes.sum()) + 1024

    def reqs():
        return [(r.arrival, Request(r.system.coords, r.system.species, r.system.box,
                                    args.req_steps, 0.01, seed=r.seed)) for r in trace]

    skip = len(trace) // 10

    def serve(use_graphs):
        # warm-up on a few requests (kernel loading, first-touch of the
        # workspace), then the trace on a fresh server
        srv = Server(model, slots=slots, capacity=cap, skin=1.0, use_graphs=use_graphs)
        replay(srv, [(0.0, q) for _, q in reqs()[:8]])
        srv.close()
        torch.cuda.synchronize()
        srv = Server(model, slots=slots, capacity=cap, skin=1.0, use_graphs=use_graphs)
        say(args, f"serving ({'graphs' if use_graphs else 'direct launches'})")
        with no_gc_pauses():
            rep = replay(srv, reqs())
        st = srv.stats()
        srv.close()
        lat = rep.latencies(skip=skip) * 1e3
        failed = sum(1 for r in rep.results.values() if r.error)
        return {"value": st.atom_evals / rep.wall, "rep": rep, "st": st, "lat": lat, "failed": failed}

    runs = {}
    if args.graphs in ("on", "both"):
        runs["graphs"] = serve(True)
    if args.graphs in ("off", "both"):
        runs["direct"] = serve(False)
    head = runs.get("graphs") or runs["direct"]
    rep, st, lat, value = head["rep"], head["st"], head["lat"], head["value"]

    def summary(r):
        st_ = r["st"]
        return {"value": round(r["value"], 1), "unit": "atom-evals/s",
                "latency_ms": {"p50": round(float(np.percentile(r["lat"], 50)), 3),
                               "p99": round(float(np.percentile(r["lat"], 99)), 3)},
                "iterations": int(st_.iterations),
                "host_us_per_iteration": round(st_.host_launch_s / max(st_.iterations, 1) * 1e6, 1),
                "graphs_recorded": int(st_.graph_captures), "graph_replays": int(st_.graph_replays),
                "wall_s": round(r["rep"].wall, 3), "failed_requests": r["failed"]}

    # plain: float32, one request at a time, one step per call, fresh lists
    plain = NNPModel(spec, "fp32")
    plain.reserve(int(sizes.max()), 1, cap)
    rng = np.random.default_rng(7)
    pick = sorted(rng.choice(len(trace), min(args.plain_requests, len(trace)), replace=False).tolist())
    p_atoms, p_time, p_lat = 0, 0.0, []
    for k in pick:
        r = trace[k]
        c = torch.as_tensor(r.system.coords, device=dev)
        s = torch.as_tensor(r.system.species, device=dev)
        box = r.system.box[None, :]
        offs = np.array([0, r.system.n], np.int64)
        g = torch.Generator(device=dev)
        g.manual_seed(int(r.seed))
        out = plain.energy_forces(c, s, box, offs)
        torch.cuda.synchronize()
        with no_gc_pauses():
            t0 = time.perf_counter()
            for _ in range(args.req_steps):
                plain.energy_forces(c, s, box, offs, out=out)
                torch.cuda.synchronize()
                c.add_(torch.randn(c.shape, generator=g, device=dev) * 0.01)
            dt = time.perf_counter() - t0
        p_time += dt
        p_atoms += r.system.n * args.req_steps
        p_lat.append(dt * 1e3)
    plain.status()
    plain_rate = p_atoms / p_time
    offered = args.rate * args.req_steps * float(sizes.mean())
    out = {
        "metric": "energy+force atom-evals/s (serving)",
        "value": round(value, 1),
        "unit": "atom-evals/s",
        "n_gpus": 1,
        "steps": int(st.iterations),
        "warmup": 8,
        "ms_per_step": round(rep.wall / max(st.iterations, 1) * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-mlp/f32-aev",
        "data": "synthetic",
        "config": {"workload": f"serving: {len(trace)} requests, Poisson {args.rate:g}/s, "
                               f"log-uniform 20-5000 atoms (half water boxes, half solutes), "
                               f"{args.req_steps} random-walk steps each",
                   "mean_atoms": round(float(sizes.mean()), 1),
                   "offered_atom_evals_per_s": round(offered, 1),
                   "form": "native continuous batching, persistent lists (1 A skin), "
                           "two iterations in flight, "
                           + ("iterations replayed from graphs recorded per capacity bucket"
                              if "graphs" in runs else "kernels launched directly"),
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3),
                       "requests": int(len(lat)), "excluded_warmup_requests": skip},
        "wall_s": round(rep.wall, 3),
        "server": {"iterations": st.iterations, "atom_evals": st.atom_evals,
                   "max_batch_seen": st.max_batch_seen, "batch_budget": st.max_batch_atoms,
                   "device_bytes": st.device_bytes, "neighbour_list_builds": st.list_builds},
        "forms": {k: summary(v) for k, v in runs.items()},
        "plain_fp32_sequential": {"value": round(plain_rate, 1), "unit": "atom-evals/s",
                                  "sample": f"{len(pick)} requests x {args.req_steps} steps",
                                  "service_ms_p50": round(float(np.percentile(p_lat, 50)), 3),
                                  "note": "service time only; at the offered load its queue grows "
                                          "without bound"},
        "speedup_vs_plain": round(value / plain_rate, 2),
    }
    print(json.dumps(out), flush=True)


def hybrid_bench(args):
    """The pair-list entry point on the 100k-atom solvated-protein box: the
    ML region is the 30,000-atom protein (V_ML(P) of the hybrid potential,
    8 networks), the caller's list is a full list of the whole box (every
    neighbour pair within the radial cutoff, built once by the library's own
    search and handed over as plain pairs).  Beside it: the same region as a
    system of its own through the library's cell search."""
    import torch
    import synth
    from paper_2207_14276_amd import NNPModel

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    full = synth.config3()
    spec = synth.make_model(3, n_ensemble=8)
    N = len(full.species)
    n_ml = 30000
    c = torch.as_tensor(full.coords, device=dev)
    sp = torch.as_tensor(full.species, device=dev)
    mask = torch.zeros(N, dtype=torch.uint8, device=dev)
    mask[:n_ml] = 1
    sub = synth.make_batch([synth.System(full.coords[:n_ml], full.species[:n_ml], full.box)])
    cs, ss = c[:n_ml].contiguous(), sp[:n_ml].contiguous()

    model = NNPModel(spec, args.precision)
    cap = size_capacity(model, sub, cs, ss, n_ml, 1)
    tuned = model.autotune(cs, ss, sub.boxes, sub.offsets)
    # the caller's list: every (i, j, image) of the whole box within 5.1 A
    model.reserve(N, 1, 128)
    cnt, ent = model.neighbors(c, sp, full.box[None, :], np.array([0, N], np.int64), capacity=128)
    model.reserve(N, 1, cap)
    valid = torch.arange(128, device=dev)[None, :] < cnt.clamp(max=128)[:, None]
    ii = torch.arange(N, device=dev, dtype=torch.int32)[:, None].expand(N, 128)[valid]
    pairs = torch.stack([ii, ent[..., 0][valid]], 1).contiguous()
    shifts = ent[..., 1:4][valid].contiguous()
    say(args, f"hybrid: N={N} region={n_ml} caller pairs={pairs.shape[0]} capacity={cap}")

    res = model.energy_forces_pairs(c, sp, full.box, pairs, shifts, mask, half=False, virial=True,
                                    atom_energy=True, check=True)
    for _ in range(args.warmup):
        model.energy_forces_pairs(c, sp, full.box, pairs, shifts, mask, half=False, out=res)
    # stage breakdown outside the timed region; the timed steps record only
    # the dominant stage's two events
    stages = probe_stages(model, lambda: model.energy_forces_pairs(c, sp, full.box, pairs, shifts, mask,
                                                                   half=False, out=res))
    dom = max(("aev_fwd", "aev_bwd", "mlp"), key=lambda k: stages.get(k, 0.0))
    st = torch.cuda.current_stream()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    model.set_timing(True, stage=dom)
    torch.cuda.synchronize()
    with no_gc_pauses():
        t0 = time.perf_counter()
        for k in range(args.steps):
            starts[k].record(st)
            model.energy_forces_pairs(c, sp, full.box, pairs, shifts, mask, half=False, out=res)
            ends[k].record(st)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    dom_ms = model.stage_timings()[dom]
    model.set_timing(False)
    model.status()
    lat = np.array([starts[k].elapsed_time(ends[k]) for k in range(args.steps)])
    value = n_ml * args.steps / wall

    # the same region through the library's own cell search
    r2 = model.energy_forces(cs, ss, sub.boxes, sub.offsets, check=True)
    torch.cuda.synchronize()
    with no_gc_pauses():
        t0 = time.perf_counter()
        for _ in range(args.steps):
            model.energy_forces(cs, ss, sub.boxes, sub.offsets, out=r2)
        torch.cuda.synchronize()
        own = n_ml * args.steps / (time.perf_counter() - t0)

    n_pairs, n_trip = pair_triplet_counts(model, sub, cs, ss)
    aev_fwd_flop = FLOP_RADIAL_FWD * n_pairs + FLOP_TRIPLET_FWD * n_trip
    aev_bwd_flop = FLOP_RADIAL_BWD * n_pairs + FLOP_TRIPLET_BWD * n_trip
    fwd_f, bwd_f = mlp_flops(spec, sub.species)
    cand = {"aev_fwd": ("alu", aev_fwd_flop, PEAK_FP32_VALU_TFLOPS),
            "aev_bwd": ("alu", aev_bwd_flop, PEAK_FP32_VALU_TFLOPS),
            "mlp": ("mfma", fwd_f + bwd_f,
                    PEAK_BF16_MFMA_TFLOPS if args.precision == "bf16" else PEAK_FP32_MFMA_TFLOPS)}
    bound, work, peak = cand[dom]
    achieved = work / (dom_ms * 1e-3) / 1e12
    kname = {"aev_fwd": "k_aev_fwd", "aev_bwd": "k_aev_bwd", "mlp": "k_gemm"}[dom]
    out = {
        "metric": "energy+force atom-evals/s (pair-list entry point, ML region)",
        "value": round(value, 1),
        "unit": "atom-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-mlp/f32-aev" if args.precision == "bf16" else "f32",
        "data": "synthetic",
        "config": {"workload": "hybrid: 30,000-atom protein region (8 networks) of the 100,002-atom "
                               "solvated box, caller's full pair list of the whole box",
                   "n_atoms": N, "n_region": n_ml, "caller_pairs": int(pairs.shape[0]),
                   "nbr_capacity": cap, "tuned_shapes": tuned, "parallelism": "single GPU"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4)},
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "roofline": {"kernel": kname if dom != "mlp" else "k_gemm (all dense layers)", "bound": bound,
                     "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4), "traffic": None,
                     "work_per_launch_flop": work, "avg_launch_ms": round(dom_ms, 4),
                     "pairs": n_pairs, "triplets": n_trip},
        "own_cell_search_same_region": {"value": round(own, 1), "unit": "atom-evals/s"},
    }
    if not args.no_cpu:
        import oracle
        om = oracle.OracleModel(spec)
        tgt = np.sort(np.random.default_rng(0).choice(n_ml, 8, replace=False))
        e_ref, f_ref = oracle.sampled(sub.coords, sub.species, sub.boxes[0], om, tgt)
        F = res.forces.cpu().numpy()
        out["error_vs_oracle"] = {
            "sample": "8 atoms of the region (local evaluation of the region alone)",
            "max_abs_dF": float(np.abs(F[tgt] - f_ref).max()),
            "max_abs_dE_atom": float(np.abs(res.atom_energy.cpu().numpy()[tgt] - e_ref).max()),
            "max_abs_F_outside_region": float(np.abs(F[n_ml:]).max())}
    print(json.dumps(out), flush=True)


def snapshots_bench(args):
    """Energy-only throughput for reweighting stored snapshots: 4,096
    snapshots of one 40-atom solute (two harmonic reference states of 2,048
    each), evaluated in one batched call per step without forces (the
    input-gradient and AEV-backward stages are skipped); beside it the same
    batch with forces, the plain float32 form (one snapshot per call, energy
    only) and the host BAR estimate on the energies."""
    import torch
    import synth
    from paper_2207_14276_amd import NNPModel
    from paper_2207_14276_amd.bar import bar_reweighted, beta_at

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    spec = synth.make_model(0)
    rng = np.random.default_rng(8)
    n_atoms, n_per = 40, 2048
    ref = synth.random_solute(rng, n_atoms, 1.2 * n_atoms ** (1 / 3), synth.CONFIG2_PROBS)
    beta = beta_at(300.0)
    ks = (20.0, 40.0)
    systems, state = [], []
    for si, k in enumerate(ks):
        sd = 1.0 / np.sqrt(beta * k)
        for _ in range(n_per):
            x = ref.coords + rng.normal(0.0, sd, size=ref.coords.shape)
            systems.append(synth.System(x.astype(np.float32), ref.species, np.zeros(3, np.float32)))
            state.append(si)
    batch = synth.make_batch(systems)
    state = np.array(state)
    N, S = batch.n_atoms, batch.n_systems
    c = torch.as_tensor(batch.coords, device=dev)
    sp = torch.as_tensor(batch.species, device=dev)
    model = NNPModel(spec, args.precision)
    cap = size_capacity(model, batch, c, sp, N, S)
    tuned = model.autotune(c, sp, batch.boxes, batch.offsets)

    def timed(forces):
        r = model.energy_forces(c, sp, batch.boxes, batch.offsets, forces=forces, check=True)
        for _ in range(args.warmup):
            model.energy_forces(c, sp, batch.boxes, batch.offsets, forces=forces, out=r)
        # stage breakdown outside the timed region; the timed steps record
        # only the dominant stage's two events (its time replaces the probe's)
        stages = probe_stages(model, lambda: model.energy_forces(c, sp, batch.boxes, batch.offsets,
                                                                 forces=forces, out=r))
        dom = max(("aev_fwd", "aev_bwd", "mlp"), key=lambda k: stages.get(k, 0.0))
        st = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        model.set_timing(True, stage=dom)
        torch.cuda.synchronize()
        with no_gc_pauses():
            t0 = time.perf_counter()
            for a, b in ev:
                a.record(st)
                model.energy_forces(c, sp, batch.boxes, batch.offsets, forces=forces, out=r)
                b.record(st)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        stages[dom] = model.stage_timings()[dom]
        model.set_timing(False)
        lat = np.array([a.elapsed_time(b) for a, b in ev])
        return r, wall, stages, lat

    r_e, wall_e, stages_e, lat_e = timed(False)
    _, wall_f, _, _ = timed(True)
    value = N * args.steps / wall_e
    e = r_e.energy.cpu().numpy().astype(np.float64)

    # plain: float32, one snapshot per call, energy only, sequential
    plain = NNPModel(spec, "fp32")
    plain.reserve(n_atoms, 1, cap)
    pick = list(range(0, S, S // 256))
    per = [(c[int(batch.offsets[k]):int(batch.offsets[k + 1])], sp[int(batch.offsets[k]):int(batch.offsets[k + 1])],
            batch.boxes[k:k + 1], np.array([0, n_atoms], np.int64)) for k in pick]
    outs = [plain.energy_forces(*q, forces=False) for q in per]
    torch.cuda.synchronize()
    with no_gc_pauses():
        t0 = time.perf_counter()
        for q, o in zip(per, outs):
            plain.energy_forces(*q, forces=False, out=o)
        torch.cuda.synchronize()
        plain_rate = len(pick) * n_atoms / (time.perf_counter() - t0)

    # host BAR on the energies (target = reference restraint + network energy)
    x_ref = ref.coords.astype(np.float64)
    Ur = np.array([[0.5 * k * ((sy.coords - x_ref) ** 2).sum() for k in ks] for sy in systems])
    ee = e - e.mean()
    a_, b_ = state == 0, state == 1
    t0 = time.perf_counter()
    dF, sF = bar_reweighted(Ur[a_, 0], Ur[a_, 1], Ur[b_, 0], Ur[b_, 1],
                            Ur[a_, 0] + ee[a_], Ur[a_, 1] + ee[a_], Ur[b_, 0] + ee[b_], Ur[b_, 1] + ee[b_],
                            beta)
    t_bar = time.perf_counter() - t0

    fwd_f, _ = mlp_flops(spec, batch.species)
    n_pairs, n_trip = pair_triplet_counts(model, batch, c, sp)
    cand = {"aev_fwd": ("alu", FLOP_RADIAL_FWD * n_pairs + FLOP_TRIPLET_FWD * n_trip, PEAK_FP32_VALU_TFLOPS),
            "mlp": ("mfma", fwd_f,
                    PEAK_BF16_MFMA_TFLOPS if args.precision == "bf16" else PEAK_FP32_MFMA_TFLOPS)}
    dom = max(cand, key=lambda k: stages_e.get(k, 0.0))
    bound, work, peak = cand[dom]
    achieved = work / (stages_e[dom] * 1e-3) / 1e12
    out = {
        "metric": "energy-only atom-evals/s (stored snapshots)",
        "value": round(value, 1),
        "unit": "atom-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_e / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-mlp/f32-aev" if args.precision == "bf16" else "f32",
        "data": "synthetic",
        "config": {"workload": "4,096 snapshots of a 40-atom solute (two harmonic reference states), "
                               "one batched energy-only call per step",
                   "n_atoms": N, "n_systems": S, "nbr_capacity": cap, "tuned_shapes": tuned,
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": round(float(np.percentile(lat_e, 50)), 4),
                       "p99": round(float(np.percentile(lat_e, 99)), 4)},
        "stages_ms": {k: round(v, 4) for k, v in stages_e.items()},
        "roofline": {"kernel": "k_aev_fwd" if dom == "aev_fwd" else "k_gemm (dense layers, forward)",
                     "bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4), "traffic": None, "work_per_launch_flop": work,
                     "avg_launch_ms": round(stages_e[dom], 4), "pairs": n_pairs, "triplets": n_trip},
        "with_forces": {"value": round(N * args.steps / wall_f, 1), "unit": "atom-evals/s"},
        "plain_fp32_per_snapshot_energy_only": {"value": round(plain_rate, 1), "unit": "atom-evals/s",
                                                "sample": f"{len(pick)} snapshots"},
        "speedup_vs_plain": round(value / plain_rate, 2),
        "bar": {"dF_kcal_mol": round(dF, 5), "sigma": round(sF, 5), "host_seconds": round(t_bar, 4),
                "note": "target = reference restraint + network energy, 2,048 snapshots per state"},
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the energy/force path "
                          "is not sharded across GPUs",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import synth
    from paper_2207_14276_amd import NNPModel

    if args.workload == "serve":
        serve_bench(args)
        return
    if args.workload == "copy":
        copy_probe(args)
        return
    if args.workload == "hybrid":
        hybrid_bench(args)
        return
    if args.workload == "snapshots":
        snapshots_bench(args)
        return
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    batch, spec, desc = workload(args.workload, args.model)
    N, S = batch.n_atoms, batch.n_systems
    say(args, f"workload {args.workload}: N={N} S={S}")
    c = torch.as_tensor(batch.coords, device=dev)
    sp = torch.as_tensor(batch.species, device=dev)

    model = NNPModel(spec, args.precision)
    cap = size_capacity(model, batch, c, sp, N, S)
    # launch shapes tuned on this batch before anything is timed
    tuned = model.autotune(c, sp, batch.boxes, batch.offsets)
    say(args, "tuned launch shapes:", tuned)
    res = model.energy_forces(c, sp, batch.boxes, batch.offsets, forces=True, virial=True,
                              atom_energy=True, check=True)
    for _ in range(args.warmup):
        model.energy_forces(c, sp, batch.boxes, batch.offsets, out=res)
    torch.cuda.synchronize()

    # The library records HIP events at its stage boundaries on the stream it
    # launches on (torch's current stream).  Each event costs a few
    # microseconds of device time, so the stage breakdown comes from a few
    # steps with every boundary recorded, outside the timed region, and the
    # timed steps record only the two events around the dominant stage: its
    # time (the roofline's) is the mean over exactly the timed steps.
    stages = probe_stages(model, lambda: model.energy_forces(c, sp, batch.boxes, batch.offsets, out=res))
    dom = max(("aev_fwd", "aev_bwd", "mlp"), key=lambda k: stages.get(k, 0.0))
    st = torch.cuda.current_stream()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    model.set_timing(True, stage=dom)
    torch.cuda.synchronize()
    with no_gc_pauses():
        t0 = time.perf_counter()
        for k in range(args.steps):
            starts[k].record(st)
            model.energy_forces(c, sp, batch.boxes, batch.offsets, out=res)
            ends[k].record(st)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    dom_ms = model.stage_timings()[dom]
    model.set_timing(False)
    model.status()
    wall = t1 - t0
    lat = np.array([starts[k].elapsed_time(ends[k]) for k in range(args.steps)])
    value = N * args.steps / wall
    say(args, f"headline {args.precision}: {wall / args.steps * 1e3:.3f} ms/step, {value:.3e} atom-evals/s")
    say(args, "stages ms:", {k: round(v, 4) for k, v in stages.items()})

    # algorithmic work
    fwd_f, bwd_f = mlp_flops(spec, batch.species)
    if args.model == "dp":
        entries, comps, kept, centres = dp_counts(model, batch, c, sp)
        aev_fwd_flop = (FLOP_DP_ENTRY_FWD * entries + FLOP_DP_COMPARE * comps + FLOP_DP_SLOT_FWD * kept
                        + FLOP_DP_CENTRE_FWD * centres)
        aev_bwd_flop = FLOP_DP_SLOT_BWD * kept + FLOP_DP_CENTRE_BWD * centres
        counts = {"entries": entries, "comparisons": comps, "kept_slots": kept}
    else:
        n_pairs, n_trip = pair_triplet_counts(model, batch, c, sp)
        aev_fwd_flop = FLOP_RADIAL_FWD * n_pairs + FLOP_TRIPLET_FWD * n_trip
        aev_bwd_flop = FLOP_RADIAL_BWD * n_pairs + FLOP_TRIPLET_BWD * n_trip
        counts = {"pairs": n_pairs, "triplets": n_trip}
    mlp_flop = fwd_f + bwd_f
    cand = {
        "aev_fwd": ("alu", aev_fwd_flop, PEAK_FP32_VALU_TFLOPS),
        "aev_bwd": ("alu", aev_bwd_flop, PEAK_FP32_VALU_TFLOPS),
        "mlp": ("mfma", mlp_flop,
                PEAK_BF16_MFMA_TFLOPS if args.precision == "bf16" else PEAK_FP32_MFMA_TFLOPS),
    }
    bound, work, peak = cand[dom]
    t_dom = dom_ms * 1e-3
    achieved = work / t_dom / 1e12
    pre = "k_dp" if args.model == "dp" else "k_aev"
    kname = {"aev_fwd": pre + "_fwd", "aev_bwd": pre + "_bwd", "mlp": "k_gemm"}[dom]
    small = bool(np.all(batch.boxes == 0)) and int(np.diff(batch.offsets).max()) <= 512
    if kname == "k_dp_bwd" and small:
        kname = "k_dp_bwd_sys"   # batches of small non-periodic systems: the per-system form
    if kname == "k_aev_bwd" and tuned.get("aev_bwd_waves", 0) >= 4:
        # a grouped form of the backward (tuned to 4-10 waves per workgroup):
        # per system for batches of small non-periodic systems, per cell on
        # grids of at least 512 cells
        if small:
            kname = "k_aev_bwd_sys"
        elif cell_count(batch, model_cutoff(spec)) >= 512:
            kname = "k_aev_bwd_cells"
    wl = args.workload + ("_dp" if args.model == "dp" else "")
    roof = {"kernel": kname if dom != "mlp" else "k_gemm (all dense layers)",
            "bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": measured_traffic(kname, wl, args.precision),
            "work_per_launch_flop": work, "avg_launch_ms": round(dom_ms, 4), **counts}
    # achieved rate of the descriptor kernels (counted work / stage time)
    work_tflops = {"desc_fwd": round(aev_fwd_flop / (stages["aev_fwd"] * 1e-3) / 1e12, 3),
                   "desc_bwd": round(aev_bwd_flop / (stages["aev_bwd"] * 1e-3) / 1e12, 3)}
    if args.model == "dp":
        # the library's stage names are those of the AEV kernels; here they
        # hold the DeepPot-style descriptor's
        stages = {("dp_" + k[4:] if k.startswith("aev_") else k): v for k, v in stages.items()}

    out = {
        "metric": "energy+force atom-evals/s",
        "value": round(value, 1),
        "unit": "atom-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-mlp/f32-aev" if args.precision == "bf16" else "f32",
        "data": "synthetic",
        "config": {"workload": desc, "n_atoms": N, "n_systems": S, "nbr_capacity": cap,
                   "tuned_shapes": tuned,
                   "form": f"batched, one call per step, {args.precision} dense layers",
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4)},
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "stages_note": f"every stage boundary recorded on {PROBE_STEPS} steps outside the timed region; "
                       f"the timed steps record only {dom}'s two events (roofline.avg_launch_ms)",
        "roofline": roof,
        "mlp_tflops": round(mlp_flop / (stages["mlp"] * 1e-3) / 1e12, 2),
        "work_tflops": work_tflops,
    }

    # plain form: float32, one system per call, sequential on one stream
    if not args.no_plain and S > 1:
        plain = NNPModel(spec, "fp32")
        plain.reserve(int(np.diff(batch.offsets).max()), 1, cap)
        offs = batch.offsets
        per_sys = []
        for k in range(S):
            a, e = int(offs[k]), int(offs[k + 1])
            per_sys.append((c[a:e], sp[a:e], batch.boxes[k:k + 1], np.array([0, e - a], np.int64)))
        outs = [plain.energy_forces(*p, forces=True) for p in per_sys]
        torch.cuda.synchronize()
        plain.status()
        tp = []
        for _ in range(max(1, args.plain_passes)):
            torch.cuda.synchronize()
            with no_gc_pauses():
                t0 = time.perf_counter()
                for p, o in zip(per_sys, outs):
                    plain.energy_forces(*p, out=o)
                torch.cuda.synchronize()
                tp.append(time.perf_counter() - t0)
        tplain = min(tp)
        out["plain_fp32_per_system"] = {"value": round(N / tplain, 1), "unit": "atom-evals/s",
                                        "ms_per_pass": round(tplain * 1e3, 3),
                                        "calls_per_pass": S}
        out["speedup_vs_plain"] = round(value / (N / tplain), 2)
        say(args, f"plain fp32 per-system: {tplain * 1e3:.2f} ms/pass, {N / tplain:.3e} atom-evals/s")

    # the same batched form with float32 dense layers: separates the gain of
    # batching from that of the precision form
    res32 = None
    if args.precision == "bf16" and not args.no_plain:
        m32 = NNPModel(spec, "fp32")
        m32.reserve(N, S, cap)
        m32.autotune(c, sp, batch.boxes, batch.offsets)
        res32 = m32.energy_forces(c, sp, batch.boxes, batch.offsets, forces=True, virial=True,
                                  atom_energy=True, check=True)
        for _ in range(args.warmup):
            m32.energy_forces(c, sp, batch.boxes, batch.offsets, out=res32)
        torch.cuda.synchronize()
        with no_gc_pauses():
            t0 = time.perf_counter()
            for _ in range(args.steps):
                m32.energy_forces(c, sp, batch.boxes, batch.offsets, out=res32)
            torch.cuda.synchronize()
            w32 = time.perf_counter() - t0
        m32.status()
        out["batched_fp32"] = {"value": round(N * args.steps / w32, 1), "unit": "atom-evals/s",
                               "ms_per_step": round(w32 / args.steps * 1e3, 4),
                               "form": "batched, one call per step, float32 dense layers"}
        out["speedup_bf16_vs_batched_fp32"] = round(value / (N * args.steps / w32), 2)
        say(args, f"batched fp32: {w32 / args.steps * 1e3:.3f} ms/step, {N * args.steps / w32:.3e} atom-evals/s")

    # error of each form against the oracle on a seeded sample of systems
    if not args.no_cpu:
        import oracle
        om = oracle.OracleModel(spec)
        rng = np.random.default_rng(0)
        pick = sorted(rng.choice(S, min(S, 8), replace=False).tolist()) if S > 1 else [0]
        if args.workload == "protein100k":
            tgt = np.sort(rng.choice(N, 8, replace=False))
            e_ref, f_ref = oracle.sampled(batch.coords, batch.species, batch.boxes[0], om, tgt)

            def errors(r):
                return {"sample": "8 atoms",
                        "max_abs_dE_atom": float(np.abs(r.atom_energy.cpu().numpy()[tgt] - e_ref).max()),
                        "max_abs_dF": float(np.abs(r.forces.cpu().numpy()[tgt] - f_ref).max())}
        else:
            ref = oracle.batch_energy_forces(batch, om, systems=pick)

            def errors(r):
                F = r.forces.cpu().numpy()
                E = r.energy.cpu().numpy()
                fe, ee = 0.0, 0.0
                for q, k in enumerate(pick):
                    a, e = int(batch.offsets[k]), int(batch.offsets[k + 1])
                    fe = max(fe, float(np.abs(F[a:e] - ref["forces"][q]).max()))
                    ee = max(ee, abs(E[k] - ref["energy"][q]) / (e - a))
                return {"sample": f"{len(pick)} systems", "max_abs_dF": fe, "max_abs_dE_per_atom": ee}
        out["error_vs_oracle"] = errors(res)
        if res32 is not None:
            out["batched_fp32"]["error_vs_oracle"] = errors(res32)

        # CPU baseline: the oracle on a bounded sample of the same workload
        t_budget = args.cpu_seconds
        if args.workload == "protein100k":
            tgt = np.arange(0, N, N // 16)[:16]
            t0 = time.perf_counter()
            oracle.sampled(batch.coords, batch.species, batch.boxes[0], om, tgt)
            dt = time.perf_counter() - t0
            cpu_rate, sample = len(tgt) / dt, f"{len(tgt)} atoms of the 100k box, local evaluation"
        else:
            done_atoms, k, t0 = 0, 0, time.perf_counter()
            order = np.random.default_rng(1).permutation(S)
            while k < S and time.perf_counter() - t0 < t_budget:
                q = int(order[k])
                a, e = int(batch.offsets[q]), int(batch.offsets[q + 1])
                oracle.energy_forces(batch.coords[a:e], batch.species[a:e], batch.boxes[q], om)
                done_atoms += e - a
                k += 1
            dt = time.perf_counter() - t0
            cpu_rate = done_atoms / dt
            sample = f"{k} of {S} systems ({done_atoms} atoms), seeded order"
        out["cpu_baseline"] = {"value": round(cpu_rate, 2), "unit": "atom-evals/s",
                               "cores": oracle.threads(), "kind": "oracle", "sample": sample,
                               "seconds": round(dt, 2), "cpu_model": cpu_model(),
                               "host_cpus": os.cpu_count()}
        say(args, f"cpu oracle: {cpu_rate:.3e} atom-evals/s on {oracle.threads()} threads")
        # the same oracle on one core, on a smaller bounded sample
        prev = oracle.set_threads(1)
        try:
            if args.workload == "protein100k":
                tgt1 = tgt[:4]
                t0 = time.perf_counter()
                oracle.sampled(batch.coords, batch.species, batch.boxes[0], om, tgt1)
                dt1 = time.perf_counter() - t0
                rate1, sample1 = len(tgt1) / dt1, f"{len(tgt1)} atoms of the 100k box, local evaluation"
            else:
                done1, k1, t0 = 0, 0, time.perf_counter()
                while k1 < S and time.perf_counter() - t0 < t_budget / 3:
                    q = int(order[k1])
                    a, e = int(batch.offsets[q]), int(batch.offsets[q + 1])
                    oracle.energy_forces(batch.coords[a:e], batch.species[a:e], batch.boxes[q], om)
                    done1 += e - a
                    k1 += 1
                dt1 = time.perf_counter() - t0
                rate1, sample1 = done1 / dt1, f"{k1} of {S} systems ({done1} atoms), seeded order"
        finally:
            oracle.set_threads(prev)
        out["cpu_baseline_1core"] = {"value": round(rate1, 2), "unit": "atom-evals/s", "cores": 1,
                                     "kind": "oracle", "sample": sample1, "seconds": round(dt1, 2)}

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
