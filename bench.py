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
# Algorithmic bytes of the step (the per-unit figures of the scope table's measurement):
# 7 B per recurrent synaptic event (int32 target + int16 weight + uint8 delay of the plain
# record layout) and 26 B per neuron per step (V, Ca and refractory state read and written,
# pending input read and cleared).  External events cost no bytes (drawn on the fly).
BYTES_PER_EVENT = 7
BYTES_PER_NEURON = 26
# The bytes this kernel's own layout needs: one 4-byte record per delivered synapse (delay
# implied by its group, target column by a rank) and 18 B per neuron (V, Ca float32 and the
# refractory counter, read and written; the input lives in LDS).
RECORD_BYTES_PER_SYNAPSE = 4
RECORD_BYTES_PER_NEURON = 18

WORKLOADS = {
    "96x96": ("PLAIN_96X96", 2000),
    "24x24": ("PLAIN_24X24", 10000),
    "2x2": ("PLAIN_2X2", 1000),
    "paper96": ("PAPER_96X96", 1000),
    "paper48": ("PAPER_48X48", 1000),
    "paper24": ("PAPER_24X24", 1000),
    "stdp24": ("STDP_24X24", 1000),
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("step.hip", "dpsnn_internal.h"):
        with open(os.path.join(ROOT, "paper_1511_09325_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_key(workload: str, delivery: str, first: int, last: int) -> str:
    return "%s/%s/steps %d-%d" % (workload, delivery, first, last)


def measured_traffic(key: str):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs of the same workload and the same timed step range, if they were taken on
    the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(key)
    except Exception:
        return None
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def _oracle_sample(sim, steps):
    """Time `steps` oracle steps (step loop only); returns (seconds, events)."""
    c0 = sim.counts()
    t0 = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t0
    c1 = sim.counts()
    return dt, (c1["e_rec"] - c0["e_rec"]) + (c1["e_ext"] - c0["e_ext"])


def cpu_baseline(sample_steps: int = 5000):
    """The CPU oracle, as it stands, on bounded samples of the same workload family (network
    construction excluded from every timing):
      * value: the 4x4 grid of the same column recipe (19,840 neurons, ~24.6M synapses),
        seed 0, `sample_steps` steps after 20 warm-up steps, one thread;
      * all_cores: the same sample with the oracle's loops over neurons and spikes on every
        host thread (OpenMP);
      * plain_24x24: the 24x24 workload's first 200 steps on every host thread, and its first
        40 steps on one thread;
      * plain_2x2_1s: the whole 2x2 workload (1000 steps), one thread."""
    import oracle
    from paper_1511_09325_amd import workloads as W
    nthreads = host_threads()
    oracle.set_threads(nthreads)
    p = W.grid(4, 4, 0)
    net = oracle.network(p)
    oracle.set_threads(1)
    sim = oracle.Sim(p, net)
    sim.step(20)
    dt, ev = _oracle_sample(sim, sample_steps)
    oracle.set_threads(nthreads)
    sim_all = oracle.Sim(p, net)
    sim_all.step(20)
    dt_all, ev_all = _oracle_sample(sim_all, sample_steps)
    assert ev_all == ev, "the oracle's result must not depend on its thread count"
    del sim, sim_all, net
    out = {"value": ev / dt, "unit": "synaptic events/s", "cores": 1, "kind": "oracle",
           "sample": "4x4 grid of the same column recipe (19,840 neurons, 24.6M synapses), "
                     "seed 0, %d steps after 20 warm-up steps, step loop only, one thread, "
                     "%.1f s" % (sample_steps, dt),
           "sim_ms_per_wall_s": sample_steps / dt,
           "host_cpu": host_cpu_model(), "host_lscpu": host_lscpu(),
           "nproc": os.cpu_count(), "threads_used": nthreads,
           "all_cores": {"value": ev_all / dt_all, "unit": "synaptic events/s",
                         "cores": nthreads, "seconds": dt_all,
                         "sim_ms_per_wall_s": sample_steps / dt_all,
                         "sample": "the same 4x4 sample, the oracle's loops on %d threads"
                                   % nthreads},
           "plain_24x24": _oracle_24x24(nthreads),
           "plain_2x2_1s": _oracle_2x2_full()}
    return out


def _oracle_24x24(nthreads: int):
    """The 24x24 workload (714,240 neurons, 885M synapses) in the oracle: its first 200 steps
    on every host thread, and its first 40 steps (a separate run from the initial state) on
    one thread."""
    import oracle
    from paper_1511_09325_amd import workloads as W
    p = W.PLAIN_24X24["params"]
    oracle.set_threads(nthreads)
    t0 = time.perf_counter()
    net = oracle.network(p)
    t_net = time.perf_counter() - t0
    sim = oracle.Sim(p, net)
    dt_all, ev_all = _oracle_sample(sim, 200)
    del sim
    oracle.set_threads(1)
    one = oracle.Sim(p, net)
    dt_one, ev_one = _oracle_sample(one, 40)
    oracle.set_threads(nthreads)
    del one, net
    return {"network_s_all_threads": t_net,
            "first_200_steps_all_threads": {"events_per_s": ev_all / dt_all, "seconds": dt_all,
                                            "cores": nthreads,
                                            "sim_ms_per_wall_s": 200 / dt_all},
            "first_40_steps_one_thread": {"events_per_s": ev_one / dt_one, "seconds": dt_one,
                                          "cores": 1, "sim_ms_per_wall_s": 40 / dt_one}}


def _oracle_2x2_full():
    """The oracle over the whole small plain workload (2x2 grid, 4,960 neurons, 1000 steps),
    one thread, step loop only."""
    import oracle
    from paper_1511_09325_amd import workloads as W
    p, steps = W.PLAIN_2X2["params"], W.PLAIN_2X2["steps"]
    oracle.set_threads(1)
    sim = oracle.Sim(p)
    dt, ev = _oracle_sample(sim, steps)
    oracle.set_threads(host_threads())
    return {"events_per_s": ev / dt, "seconds": dt, "cores": 1,
            "sim_ms_per_wall_s": steps * p["dt"] / dt}


def host_threads() -> int:
    """Host threads this process may use: OMP_NUM_THREADS when set (the host's share for the
    job), else the CPUs of its affinity mask."""
    try:
        n = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        n = 0
    if n > 0:
        return n
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


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


def host_lscpu() -> dict:
    """The host CPU as lscpu describes it (model, family, sockets, cores, caches, clocks)."""
    import subprocess
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
    except Exception:
        return {}
    keep = ("Architecture", "CPU(s)", "On-line CPU(s) list", "Vendor ID", "Model name",
            "CPU family", "Model", "Stepping", "Thread(s) per core", "Core(s) per socket",
            "Socket(s)", "CPU max MHz", "CPU min MHz", "BogoMIPS", "L1d cache", "L2 cache",
            "L3 cache", "NUMA node(s)", "Hypervisor vendor", "Virtualization type")
    out = {}
    for line in txt.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            if k.strip() in keep:
                out[k.strip()] = v.strip()
    return out


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


def models_leg(torch, warmup=50):
    """The neuron-model variants on the 24x24 grid (1 s each, the default launch): LIF with a
    second (sodium-dependent) AHP variable and Izhikevich RS/FS neurons, beside the plain LIF
    network of the same grid over the same steps."""
    from paper_1511_09325_amd import Simulation
    from paper_1511_09325_amd import workloads as W
    out = {}
    for key, preset in (("plain_lif", dict(W.PLAIN_24X24, steps=1000)),
                        ("sodium_ahp", W.SODIUM_AHP_24X24), ("izhikevich", W.IZHIKEVICH_24X24)):
        p, steps = preset["params"], preset["steps"]
        sim = Simulation(p)
        sim.step(warmup)
        sim.sync()
        t, ev, spk = _timed_run(sim, steps - warmup, torch)
        out[key] = {"workload": preset["name"] if key != "plain_lif"
                    else "24x24, LIF with the calcium AHP, 1 s",
                    "timed_steps": "%d-%d" % (warmup, steps - 1),
                    "ms_per_step": t * 1e3 / (steps - warmup), "events_per_s": ev / t,
                    "sim_ms_per_wall_s": (steps - warmup) * p["dt"] / t,
                    "mean_rate_hz": spk / (sim.n_neurons * (steps - warmup) * p["dt"] * 1e-3)}
        sim.close()
        del sim
    torch.cuda.empty_cache()
    return out


def stdp_leg(torch, warmup=50):
    """The 24x24 grid with spike-timing-dependent plasticity on (1 s, default launch) beside
    the same grid without it, over the same steps: the cost of the depression inside the
    delivery and of the potentiation kernel."""
    from paper_1511_09325_amd import Simulation
    from paper_1511_09325_amd import workloads as W
    out = {}
    for key, preset in (("static", dict(W.PLAIN_24X24, steps=1000)), ("stdp", W.STDP_24X24)):
        p, steps = preset["params"], preset["steps"]
        t0 = time.time()
        sim = Simulation(p)
        sim.sync()
        gen = time.time() - t0
        sim.step(warmup)
        sim.sync()
        t, ev, spk = _timed_run(sim, steps - warmup, torch)
        out[key] = {"workload": preset["name"] if key == "stdp"
                    else "24x24, LIF with the calcium AHP, static weights, 1 s",
                    "timed_steps": "%d-%d" % (warmup, steps - 1), "setup_s": gen,
                    "device_bytes": sim.device_bytes,
                    "ms_per_step": t * 1e3 / (steps - warmup), "events_per_s": ev / t,
                    "sim_ms_per_wall_s": (steps - warmup) * p["dt"] / t,
                    "mean_rate_hz": spk / (sim.n_neurons * (steps - warmup) * p["dt"] * 1e-3)}
        sim.close()
        del sim
    out["stdp_over_static"] = out["stdp"]["ms_per_step"] / out["static"]["ms_per_step"]
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
        return float(loss.detach())

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


def plain_leg(torch, workload: str, steps, warmup: int, delivery: str = "arrival",
              block: int = 0, tile=(0, 0), gather: int = 0, with_traffic: bool = True):
    """One plain workload on the GPU: the network is generated, the untimed first part of the
    workload's run is stepped (settle, then warm-up), and the last `steps` steps of the run
    are timed -- so a short timed window measures the state the named run ends in, not its
    start-up transient.  Returns the leg's figures with the roofline of its dominant kernel."""
    from paper_1511_09325_amd import DELIVERY_ARRIVAL, DELIVERY_PUSH, Simulation
    from paper_1511_09325_amd import workloads as W
    preset_name, run_steps = WORKLOADS[workload]
    preset = getattr(W, preset_name)
    p = preset["params"]
    K = steps if steps is not None else max(1, run_steps - warmup)
    settle = max(0, run_steps - warmup - K)
    first, last = settle + warmup, settle + warmup + K - 1
    total = max(run_steps, last + 1)
    log("generating %s on the GPU" % preset["name"])
    t0 = time.perf_counter()
    sim = Simulation(p, delivery=DELIVERY_ARRIVAL if delivery == "arrival" else DELIVERY_PUSH,
                     block=block, tile=tile, gather_steps=gather)
    launch = sim.get_launch()
    sim.sync()
    t_gen = time.perf_counter() - t0
    log("generated %d neurons, %d synapses in %.1f s (%.1f GB on device)"
        % (sim.n_neurons, sim.n_synapses, t_gen, sim.device_bytes / 1e9))
    if settle:
        sim.step(settle)
        sim.sync()
        log("settled %d untimed steps" % settle)
    sim.step(warmup)
    sim.sync()
    log("warm-up %d steps done" % warmup)
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
    sim.set_timing(False)
    log("timed steps %d-%d in %.1f ms" % (first, last, wall_ms))

    e_rec = s1["e_rec"] - s0["e_rec"]
    e_ext = s1["e_ext"] - s0["e_ext"]
    spikes = s1["spikes"] - s0["spikes"]
    streamed = s1["streamed"] - s0["streamed"]
    delivered = s1["delivered"] - s0["delivered"]
    secs = wall_ms / 1e3
    N = sim.n_neurons
    if delivery == "push":
        # the push form's delivery kernel streams the synapses, its update kernel the neurons
        kern, dom_name, events = tm["deliver"], "k_deliver_push", streamed
        per_launch = BYTES_PER_EVENT * events / K
        rec_per_launch = RECORD_BYTES_PER_SYNAPSE * streamed / K
    else:
        # arrival form: one fused launch per step gathers the step's arriving synapses and
        # updates every neuron
        kern, dom_name = tm["update"], "k_step_tile"
        if p.get("stdp"):  # the step's launches also hold the potentiation kernel
            dom_name = "k_step_tile + k_stdp_post"
        per_launch = (BYTES_PER_EVENT * delivered + BYTES_PER_NEURON * N * K) / K
        rec_per_launch = (RECORD_BYTES_PER_SYNAPSE * delivered + RECORD_BYTES_PER_NEURON * N * K) / K
    dom_ms = kern["ms"] / max(kern["launches"], 1)
    achieved = per_launch / (dom_ms * 1e-3) / 1e9
    key = traffic_key(workload, delivery, first, last)
    traffic = measured_traffic(key) if with_traffic else None
    roof = {"bound": "hbm", "kernel": dom_name, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_source": ("profiles/traffic.json [%s]" % key) if traffic else None,
            "avg_launch_ms": dom_ms, "launches": kern["launches"],
            "algorithmic_bytes_per_launch": per_launch,
            "bytes_per_unit": "%d B per recurrent event delivered + %d B per neuron per step"
                              % (BYTES_PER_EVENT, BYTES_PER_NEURON),
            "events_delivered_per_launch": delivered / K,
            "synapse_records_read_per_launch": streamed / K,
            "record_layout": {"bytes_per_launch": rec_per_launch,
                              "achieved": rec_per_launch / (dom_ms * 1e-3) / 1e9,
                              "frac": rec_per_launch / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "bytes_per_unit": "%d B per delivered synapse record + %d B per "
                                                "neuron per step (the kernel's own layout)"
                                                % (RECORD_BYTES_PER_SYNAPSE, RECORD_BYTES_PER_NEURON)}}
    if traffic:
        roof["traffic_over_algorithmic"] = traffic / per_launch
        roof["traffic_over_record_layout"] = traffic / rec_per_launch
    out = {"workload": "%s; timed steps %d-%d of the %d-step run"
                       % (preset["name"], first, last, total),
           "grid": workload, "neurons": N, "synapses": sim.n_synapses, "dt_ms": p["dt"],
           "settle_steps": settle, "first_timed_step": first, "last_timed_step": last,
           "delivery": delivery, "block": launch["block"], "tile": "%dx%d" % launch["tile"],
           "gather_steps": launch["gather_steps"],
           "steps": K, "ms_per_step": wall_ms / K, "events_per_s": (e_rec + e_ext) / secs,
           "sim_ms_per_wall_s": K * p["dt"] / secs, "recurrent_events_per_s": e_rec / secs,
           "external_events_per_s": e_ext / secs,
           "mean_rate_hz": spikes / (N * K * p["dt"] * 1e-3), "generation_s": t_gen,
           "roofline": roof}
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps, the last of the workload's run (default: all of the run "
                         "after the warm-up)")
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
    ap.add_argument("--no-small-grids", action="store_true")
    ap.add_argument("--no-models", action="store_true")
    ap.add_argument("--no-paper-recipe", action="store_true")
    ap.add_argument("--no-stdp", action="store_true")
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
    tile = (0, 0) if args.tile == "auto" else tuple(int(x) for x in args.tile.split("x"))
    main_leg = plain_leg(torch, args.workload, args.steps, args.warmup, args.delivery,
                         args.block, tile, args.gather)
    roof = main_leg.pop("roofline")
    copy_gbs = device_copy_gbs(torch)
    roof["device_copy_gbs"] = copy_gbs
    roof["frac_of_copy"] = roof["achieved"] / copy_gbs
    K = main_leg["steps"]
    out = {
        "metric": "synaptic events/s (recurrent + external) and sim-ms per wall-s",
        "value": main_leg["events_per_s"],
        "unit": "synaptic events/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "int32 input, f32 state",
        "data": "synthetic (seeded network and Poisson input of the column recipe)",
        "config": dict({k: main_leg[k] for k in (
            "workload", "grid", "neurons", "synapses", "dt_ms", "settle_steps",
            "first_timed_step", "last_timed_step", "delivery", "block", "tile",
            "gather_steps")}, parallelism="single GPU"),
        "sim_ms_per_wall_s": main_leg["sim_ms_per_wall_s"],
        "recurrent_events_per_s": main_leg["recurrent_events_per_s"],
        "external_events_per_s": main_leg["external_events_per_s"],
        "mean_rate_hz": main_leg["mean_rate_hz"],
        "generation_s": main_leg["generation_s"],
        "roofline": roof,
    }
    if not args.no_small_grids and args.workload == "96x96":
        log("small-grid legs: the whole 24x24 (10 s) and 2x2 (1 s) workloads")
        out["small_grids"] = {w: plain_leg(torch, w, None, args.warmup) for w in ("24x24", "2x2")}
    if not args.no_paper_recipe and args.workload == "96x96":
        log("paper-recipe leg: the paper's own column recipe on the 96x96 grid")
        out["paper_recipe"] = plain_leg(torch, "paper96", 500, args.warmup)
    if not args.no_models and args.workload == "96x96":
        log("neuron-model legs: 24x24 with the sodium AHP and with Izhikevich neurons")
        out["models"] = models_leg(torch)
    if not args.no_stdp and args.workload == "96x96":
        log("plasticity leg: 24x24 with STDP on, beside static weights")
        out["stdp"] = stdp_leg(torch)
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
        log("timing the CPU oracle samples")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
