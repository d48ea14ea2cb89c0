#!/usr/bin/env python
"""bench.py -- throughput of the DPSNN per-1 ms step on one MI355X.

Default workload: the plain 96x96 grid of 1240-neuron columns (11,427,840 neurons, about
14.2G recurrent synapses generated on the GPU), 2 s simulated at dt = 1 ms, synthetic and
seeded.  One "step" is one 1 ms step of the whole network: every neuron updated, every
delayed spike delivered.

Prints ONE JSON line.  `value` is synaptic events per second (recurrent events -- the
outgoing synapses of every emitted spike -- plus external Poisson arrivals, the paper's
event definition), with the network resident in HBM before the timed region starts.
`roofline` prices the dominant kernel (the fused gather + update step kernel) against
HBM bandwidth, with its duration measured by HIP events around every launch on the
simulation's stream.  `cpu_baseline` times the plain CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_SYNAPSE = 4       # one uint32 record: target index in column (16 b) + weight (16 b)
BYTES_PER_NEURON = 18       # V, Ca (float32) and refractory counter (uint8), read and written

WORKLOADS = {
    "96x96": ("PLAIN_96X96", 2000),
    "24x24": ("PLAIN_24X24", 10000),
    "2x2": ("PLAIN_2X2", 1000),
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("step.hip", "dpsnn_internal.h"):
        with open(os.path.join(ROOT, "paper_1511_09325_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, delivery: str):
    """HBM bytes per launch from committed rocprofv3 FETCH_SIZE / WRITE_SIZE runs, if they
    were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get("%s/%s" % (workload, delivery))
    except Exception:
        return None
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(sample_steps: int = 5000):
    """The CPU oracle, as it stands, on a bounded sample of the same workload family: the
    4x4 grid of the same column recipe (19,840 neurons, ~24.6M synapses), seed 0; only its
    step loop is timed (network construction excluded); one thread."""
    import oracle
    from paper_1511_09325_amd import workloads as W
    p = W.grid(4, 4, 0)
    net = oracle.network(p)
    sim = oracle.Sim(p, net)
    sim.step(20)
    c0 = sim.counts()
    t0 = time.perf_counter()
    sim.step(sample_steps)
    dt = time.perf_counter() - t0
    c1 = sim.counts()
    ev = (c1["e_rec"] - c0["e_rec"]) + (c1["e_ext"] - c0["e_ext"])
    return {"value": ev / dt, "unit": "synaptic events/s", "cores": 1, "kind": "oracle",
            "sample": "4x4 grid of the same column recipe (19,840 neurons, %d synapses), "
                      "seed 0, %d steps after 20 warm-up steps, step loop only, %.1f s"
                      % (len(net[1]), sample_steps, dt),
            "sim_ms_per_wall_s": sample_steps / dt,
            "host_cpu": host_cpu_model(), "host_threads": os.cpu_count(),
            "plain_2x2_1s": _oracle_2x2_full()}


def _oracle_2x2_full():
    """The oracle over the whole small plain workload (2x2 grid, 4,960 neurons, 1000 steps),
    one thread, step loop only."""
    import oracle
    from paper_1511_09325_amd import workloads as W
    p, steps = W.PLAIN_2X2["params"], W.PLAIN_2X2["steps"]
    sim = oracle.Sim(p)
    t0 = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t0
    c = sim.counts()
    return {"events_per_s": (c["e_rec"] + c["e_ext"]) / dt, "seconds": dt,
            "sim_ms_per_wall_s": steps * p["dt"] / dt}


def host_cpu_model() -> str:
    """The host CPU's model name as /proc/cpuinfo gives it (empty if unavailable)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def device_copy_gbs(torch, mib: int = 2048, reps: int = 10) -> float:
    """Bandwidth of a plain device-to-device copy (bytes read + written per second), the
    practical HBM ceiling the roofline fraction is also quoted against."""
    n = (mib << 20) // 4
    src = torch.empty(n, dtype=torch.int32, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * (mib << 20) * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


def _timed_run(sim, steps, torch):
    """Run `steps` steps on the simulation's stream; returns (seconds, events, spikes)."""
    s0 = [sim.stats(n) for n in range(sim.n_nets)]
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    sim.sync()
    s1 = [sim.stats(n) for n in range(sim.n_nets)]
    ev = sum((b["e_rec"] - a["e_rec"]) + (b["e_ext"] - a["e_ext"]) for a, b in zip(s0, s1))
    spk = sum(b["spikes"] - a["spikes"] for a, b in zip(s0, s1))
    return e0.elapsed_time(e1) / 1e3, ev, spk


def batched_leg(torch, steps=1000, warmup=50, graph_steps=50):
    """64 independent networks (seeds 0-63, grid sides 2..8, external rates 2-6 Hz), 1 s
    each: one simulation stepping all of them with one launch per step, against the 64
    networks run one after the other as plain simulations, on the same GPU."""
    from paper_1511_09325_amd import Simulation
    from paper_1511_09325_amd import workloads as W
    nets = W.batched_networks(64, 0)
    sim = Simulation(nets)
    sim.set_launch(graph_steps=graph_steps)
    sim.step(warmup)
    tuned = sim.autotune(window=graph_steps)
    t_b, ev_b, spk_b = _timed_run(sim, steps, torch)
    n_neurons, n_syn = sim.n_neurons, sim.n_synapses
    del sim
    t_s, ev_s = 0.0, 0
    for p in nets:
        one = Simulation(p)
        one.set_launch(graph_steps=graph_steps)
        one.step(warmup)
        t, ev, _ = _timed_run(one, steps, torch)
        t_s += t
        ev_s += ev
        del one
    assert ev_s == ev_b, "batched and sequential runs must deliver the same events"
    return {"workload": "64 networks, seeds 0-63, grids 2x2..8x8, ext 2-6 Hz, %d steps each"
                        % steps,
            "neurons": n_neurons, "synapses": n_syn, "launch": tuned,
            "batched_events_per_s": ev_b / t_b, "sequential_events_per_s": ev_s / t_s,
            "batched_sim_ms_per_wall_s": steps / t_b, "speedup_vs_sequential": t_s / t_b,
            "mean_rate_hz": spk_b / (n_neurons * steps * 1e-3)}


def rate_matched_leg(torch, steps=1000, warmup=50):
    """The 96x96 grid with inhibitory weights -N(1.2, 0.12) mV (a few Hz instead of the tens
    of Hz of the literal parameters), same launch defaults: the low-rate end of the step."""
    from paper_1511_09325_amd import Simulation
    from paper_1511_09325_amd import workloads as W
    preset = W.PLAIN_96X96_RATE_MATCHED
    p = preset["params"]
    sim = Simulation(p)
    sim.step(warmup)
    sim.sync()
    t, ev, spk = _timed_run(sim, steps, torch)
    out = {"workload": preset["name"], "steps": steps, "ms_per_step": t * 1e3 / steps,
           "events_per_s": ev / t, "sim_ms_per_wall_s": steps * p["dt"] / t,
           "mean_rate_hz": spk / (sim.n_neurons * steps * p["dt"] * 1e-3)}
    del sim
    torch.cuda.empty_cache()
    return out


def fwd_bwd_leg(torch, iters=3):
    """Forward+backward on the 4x4 grid (19,840 neurons), 500 ms, checkpoints every 50
    steps: loss = mean over columns of (rate - target)^2 with seeded U(2, 8) Hz targets,
    surrogate-gradient backward to the float32 weights, tau_m and g_AHP.  Timed per
    training iteration (rewind, forward, rates, loss, backward), against the plain forward
    of the same network on the same GPU."""
    from paper_1511_09325_amd import Simulation
    from paper_1511_09325_amd import sim as S
    from paper_1511_09325_amd import workloads as W
    preset = W.FWD_BWD_4X4
    p, T, K = preset["params"], preset["steps"], preset["ckpt_every"]
    plain = Simulation(p)
    plain.save(0)
    plain.step(T)                       # warm-up pass
    plain.restore(0)
    t_plain, ev_plain, _ = _timed_run(plain, T, torch)
    del plain
    sim = Simulation(p, train_mode=True, ckpt_every=K, surrogate_beta=5.0)
    target = torch.tensor(W.target_rates(sim.n_cols, 1), device="cuda")
    w = sim.get_weights().clone().requires_grad_(True)
    tau = torch.tensor(p["tau_m"], dtype=torch.float64, requires_grad=True)
    g = torch.tensor(p["g_ahp"], dtype=torch.float64, requires_grad=True)

    def iteration():
        for x in (w, tau, g):
            x.grad = None
        rates = S.column_rates(sim, w, tau, g, T)
        loss = ((rates - target) ** 2).mean()
        loss.backward()
        return float(loss)

    iteration()                          # warm-up
    torch.cuda.synchronize()
    times, losses = [], []
    for _ in range(iters):
        t0 = time.perf_counter()
        losses.append(iteration())
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    st = sim.stats()
    t_it = min(times)
    return {"workload": preset["name"] + ", checkpoints every %d steps" % K,
            "neurons": sim.n_neurons, "synapses": sim.n_synapses, "steps": T,
            "loss": losses[-1], "grad_w_norm": float(w.grad.norm()),
            "grad_tau_m": float(tau.grad), "grad_g_ahp": float(g.grad),
            "plain_forward_ms": t_plain * 1e3, "fwd_bwd_ms": t_it * 1e3,
            "fwd_bwd_over_plain": t_it / t_plain,
            "plain_events_per_s": ev_plain / t_plain,
            "fwd_bwd_events_per_s": (st["e_rec"] + st["e_ext"]) / t_it,
            "fwd_bwd_sim_ms_per_wall_s": T * p["dt"] / t_it}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's)")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="96x96", choices=sorted(WORKLOADS))
    ap.add_argument("--delivery", default="arrival", choices=["arrival", "push"])
    ap.add_argument("--block", type=int, default=0, help="workgroup size (0: library default)")
    ap.add_argument("--tile", default="auto", help="arrival tile of target columns, e.g. 4x4")
    ap.add_argument("--gather", type=int, default=0,
                    help="arrival form: steps gathered per pass (0: library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-fwd-bwd", action="store_true")
    ap.add_argument("--no-rate-matched", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first copy a buffer of this many MiB once (a reference kernel of known "
                         "traffic for hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the path is single-GPU by design "
              "(no sharding, no collectives); --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1511_09325_amd import DELIVERY_ARRIVAL, DELIVERY_PUSH, Simulation
    from paper_1511_09325_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration_mib:
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copied %d MiB for counter calibration" % args.copy_calibration_mib)
        del src, dst
    preset_name, default_steps = WORKLOADS[args.workload]
    preset = getattr(W, preset_name)
    p = preset["params"]
    K = args.steps if args.steps is not None else default_steps
    delivery = DELIVERY_ARRIVAL if args.delivery == "arrival" else DELIVERY_PUSH

    log("generating %s on the GPU" % preset["name"])
    t0 = time.perf_counter()
    tile = (0, 0) if args.tile == "auto" else tuple(int(x) for x in args.tile.split("x"))
    sim = Simulation(p, delivery=delivery, block=args.block, tile=tile, gather_steps=args.gather)
    launch = sim.get_launch()
    sim.sync()
    t_gen = time.perf_counter() - t0
    log("generated %d neurons, %d synapses in %.1f s (%.1f GB on device)"
        % (sim.n_neurons, sim.n_synapses, t_gen, sim.device_bytes / 1e9))

    sim.step(args.warmup)
    sim.sync()
    log("warm-up %d steps done" % args.warmup)
    s0 = sim.stats()
    sim.set_timing(True)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    sim.step(K)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall_ms = ev0.elapsed_time(ev1)
    sim.sync()
    tm = sim.timing()
    s1 = sim.stats()
    log("timed %d steps in %.1f ms" % (K, wall_ms))

    e_rec = s1["e_rec"] - s0["e_rec"]
    e_ext = s1["e_ext"] - s0["e_ext"]
    spikes = s1["spikes"] - s0["spikes"]
    streamed = s1["streamed"] - s0["streamed"]
    delivered = s1["delivered"] - s0["delivered"]
    secs = wall_ms / 1e3
    value = (e_rec + e_ext) / secs

    kern = tm["update"]
    dom_ms = kern["ms"] / max(kern["launches"], 1)
    if args.delivery == "push":
        # in the push form the delivery kernel streams the synapses; the update kernel the neurons
        dk = tm["deliver"]
        dom_ms = dk["ms"] / max(dk["launches"], 1)
        bytes_per_launch = BYTES_PER_SYNAPSE * streamed / K
        dom_name = "k_deliver_push"
    else:
        bytes_per_launch = (BYTES_PER_SYNAPSE * delivered + BYTES_PER_NEURON * sim.n_neurons * K) / K
        dom_name = "k_step_tile"
    achieved = bytes_per_launch / (dom_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload, args.delivery)
    copy_gbs = device_copy_gbs(torch)

    out = {
        "metric": "synaptic events/s (recurrent + external) and sim-ms per wall-s",
        "value": value,
        "unit": "synaptic events/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": wall_ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32 input, f32 state",
        "data": "synthetic (seeded network and Poisson input of the column recipe)",
        "config": {"workload": preset["name"], "grid": args.workload, "neurons": sim.n_neurons,
                   "synapses": sim.n_synapses, "dt_ms": p["dt"], "delivery": args.delivery,
                   "block": launch["block"], "tile": "%dx%d" % launch["tile"],
                   "gather_steps": launch["gather_steps"],
                   "parallelism": "single GPU"},
        "sim_ms_per_wall_s": K * p["dt"] / secs,
        "recurrent_events_per_s": e_rec / secs,
        "external_events_per_s": e_ext / secs,
        "mean_rate_hz": spikes / (sim.n_neurons * K * p["dt"] * 1e-3),
        "generation_s": t_gen,
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "avg_launch_ms": dom_ms,
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "synapse_records_read_per_launch": streamed / K,
                     "device_copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
    }
    del sim
    torch.cuda.empty_cache()
    if not args.no_batched:
        log("batched leg: 64 networks, one launch per step, vs 64 sequential runs")
        out["batched"] = batched_leg(torch)
    if not args.no_rate_matched and args.workload == "96x96":
        log("rate-matched leg: 96x96 with stronger inhibition")
        out["rate_matched"] = rate_matched_leg(torch)
    if not args.no_fwd_bwd:
        log("forward+backward leg: 4x4, 500 steps, vs the plain forward")
        out["fwd_bwd"] = fwd_bwd_leg(torch)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
