"""Python front end of libdpsnn: one Simulation object per sim_t handle.

Argument marshalling only -- every step of the simulation runs in the HIP kernels behind
the C ABI.  PyTorch supplies the HIP stream (its current stream) and, in train mode, the
device tensors that carry weights and gradients.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


def _stream_ptr(stream):
    if stream is not None:
        return C.c_void_p(stream)
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return C.c_void_p(None)


def make_config(params: dict | list[dict], *, delivery: int = L.DELIVERY_AUTO, block: int = 0,
                tile: tuple[int, int] = (0, 0), record_steps: int = 0, raster_capacity: int = 0,
                train_mode: bool = False, ckpt_every: int = 50, surrogate_beta: float = 5.0):
    """sim_config_t from one parameter dict, or a list of them (batched form: all share the
    column recipe of the first; grid shape, seed and external rate are per network)."""
    plist = params if isinstance(params, list) else [params]
    p0 = plist[0]
    nets = (L.SimNet * len(plist))()
    for n, p in enumerate(plist):
        nets[n].rows, nets[n].cols = int(p["rows"]), int(p["cols"])
        nets[n].seed = int(p["seed"])
        nets[n].ext_rate_hz = float(p["ext_rate_hz"])
    c = L.SimConfig()
    for name in ("npc", "n_exc", "d_min", "d_max", "t_ref", "ext_syn", "neuron_model",
                 "conn_kernel", "stdp"):
        setattr(c, name, int(p0[name]))
    for name in ("p_own", "p_remote", "decay_um", "spacing_um", "we_mu", "we_sigma", "wi_mu",
                 "wi_sigma", "tau_m", "theta", "v_reset", "tau_ca", "ca_inc", "g_ahp", "dt",
                 "j_ext", "tau_na", "na_inc", "g_na", "izh_a_e", "izh_b_e", "izh_c_e",
                 "izh_d_e", "izh_a_i", "izh_b_i", "izh_c_i", "izh_d_i", "izh_vpeak",
                 "lateral_amp", "lateral_sigma_um", "lateral_cutoff", "stdp_tau_plus",
                 "stdp_tau_minus", "stdp_a_plus", "stdp_a_minus", "stdp_w_max"):
        setattr(c, name, float(p0[name]))
    c.n_nets = len(plist)
    c.nets = C.cast(nets, C.POINTER(L.SimNet))
    c.delivery, c.block = int(delivery), int(block)
    c.tile_x, c.tile_y = int(tile[0]), int(tile[1])
    c.record_steps, c.raster_capacity = int(record_steps), int(raster_capacity)
    c.train_mode, c.ckpt_every = int(bool(train_mode)), int(ckpt_every)
    c.surrogate_beta = float(surrogate_beta)
    return c, nets


def tune_tiling(params, settle: int = 50, window: int = 100, **options):
    """sim_tune_tiling: the native tiling (tile_x, tile_y) measured fastest for this
    configuration, and its time per step in ms.  Builds one simulation per admissible shape in
    turn (the device memory of one at a time)."""
    cfg, _nets = make_config(params, **options)
    tx, ty, ms = C.c_int32(), C.c_int32(), C.c_double()
    L.check(L.lib().sim_tune_tiling(C.byref(cfg), int(settle), int(window), C.byref(tx),
                                    C.byref(ty), C.byref(ms)), None)
    return (tx.value, ty.value), ms.value


def query_sizes(params, **options) -> dict:
    """sim_query_sizes: the device memory of the four caller-ownable regions (bytes) and the
    state region's offsets, for the configuration make_config(params, **options) builds."""
    cfg, _nets = make_config(params, **options)
    sz = L.SimSizes()
    L.check(L.lib().sim_query_sizes(C.byref(cfg), C.byref(sz)), None)
    return {name: getattr(sz, name) for name, _ in L.SimSizes._fields_}


class Simulation:
    def __init__(self, params, *, delivery: int = L.DELIVERY_AUTO, block: int = 0,
                 tile: tuple[int, int] = (0, 0), record_steps: int = 0,
                 raster_capacity: int | None = None, train_mode: bool = False,
                 ckpt_every: int = 50, surrogate_beta: float = 5.0, gather_steps: int = 0,
                 stream=None, torch_buffers=()):
        """torch_buffers: names of the regions ("synapses", "index", "state", "history") whose
        device memory torch allocates and owns (sized by sim_query_sizes); the rest the
        library allocates."""
        self.params = params if isinstance(params, list) else [params]
        if raster_capacity is None:
            n = sum(p["rows"] * p["cols"] * p["npc"] for p in self.params)
            raster_capacity = max(1, int(record_steps * n * 0.2)) if record_steps else 0
        options = dict(delivery=delivery, block=block, tile=tile, record_steps=record_steps,
                       raster_capacity=raster_capacity, train_mode=train_mode,
                       ckpt_every=ckpt_every, surrogate_beta=surrogate_beta)
        cfg, self._nets = make_config(params, **options)
        self._cfg = cfg
        self.train_mode = bool(train_mode)
        self.lib = L.lib()
        self.buffers, self.sizes, bufs = {}, None, None
        if torch_buffers:
            import torch
            self.sizes = query_sizes(params, **options)
            bufs = L.SimBuffers()
            for name, size_field in L.REGIONS:
                if name in torch_buffers:
                    t = torch.empty(int(self.sizes[size_field]), dtype=torch.uint8, device="cuda")
                    self.buffers[name] = t
                    setattr(bufs, name, C.c_void_p(t.data_ptr()))
                    setattr(bufs, size_field, t.numel())
            unknown = set(torch_buffers) - {n for n, _ in L.REGIONS}
            if unknown:
                raise ValueError("unknown regions %s" % sorted(unknown))
        h = C.c_void_p()
        L.check(self.lib.sim_create(C.byref(cfg), C.byref(bufs) if bufs is not None else None,
                                    _stream_ptr(stream), C.byref(h)), None)
        self.h = h
        info = L.SimInfo()
        L.check(self.lib.sim_get_info(self.h, C.byref(info)), self.h)
        self.n_nets = info.n_nets
        self.n_cols = info.n_cols
        self.n_neurons = info.n_neurons
        self.n_synapses = info.n_synapses
        self.ring_slots = info.ring_slots
        self.device_bytes = info.device_bytes
        self.caller_bytes = info.caller_bytes
        self.record_steps = record_steps
        if gather_steps:
            self.set_launch(gather_steps=gather_steps)

    def state_tensors(self):
        """(V, Ca, refractory counters) of all networks as torch views of the caller-owned state
        region (torch_buffers must include "state"); read them between synchronising calls."""
        t = self.buffers["state"]
        n = self.n_neurons
        v0, c0, r0 = (int(self.sizes[k]) for k in ("state_v_offset", "state_ca_offset",
                                                   "state_ref_offset"))
        import torch
        return (t[v0:v0 + 4 * n].view(torch.float32), t[c0:c0 + 4 * n].view(torch.float32),
                t[r0:r0 + n])

    # -- lifetime -------------------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.sim_destroy(self.h)
            self.h = None
        self.buffers = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stepping -------------------------------------------------------------------------
    def step(self, n: int = 1):
        L.check(self.lib.sim_step(self.h, int(n)), self.h)

    def sync(self):
        L.check(self.lib.sim_sync(self.h), self.h)

    @property
    def now(self) -> int:
        return self.lib.sim_now(self.h)

    # -- outputs --------------------------------------------------------------------------
    def net_neurons(self, net: int = 0) -> int:
        p = self.params[net]
        return p["rows"] * p["cols"] * p["npc"]

    def read_spikes(self, net: int = 0, t0: int = 0, t1: int | None = None):
        """List (one array per step) of ascending network-local spike ids (views of one
        buffer that holds the whole range)."""
        if t1 is None:
            t1 = min(self.now, self.record_steps)
        off = np.zeros(t1 - t0 + 1, np.int64)
        n = C.c_int64(0)
        rc = self.lib.sim_read_spikes(self.h, net, t0, t1, off.ctypes.data_as(C.POINTER(C.c_int64)),
                                      None, 0, C.byref(n))
        if rc not in (L.OK, L.ETRUNC):
            L.check(rc, self.h)
        ids = np.empty(max(n.value, 1), np.int32)
        L.check(self.lib.sim_read_spikes(self.h, net, t0, t1,
                                         off.ctypes.data_as(C.POINTER(C.c_int64)),
                                         ids.ctypes.data_as(C.POINTER(C.c_int32)), ids.size,
                                         C.byref(n)), self.h)
        return [ids[off[q]:off[q + 1]] for q in range(t1 - t0)]

    def stats(self, net: int = 0) -> dict:
        s = L.SimStats()
        L.check(self.lib.sim_get_stats(self.h, net, C.byref(s)), self.h)
        return {"steps": s.steps, "spikes": s.spikes, "e_rec": s.events_recurrent,
                "e_ext": s.events_external, "streamed": s.synapses_streamed,
                "delivered": s.synapses_delivered}

    def state(self, net: int = 0, pend: bool = True) -> dict:
        n = self.net_neurons(net)
        v = np.zeros(n, np.float32)
        ca = np.zeros(n, np.float32)
        ref = np.zeros(n, np.uint8)
        pd = np.zeros((self.ring_slots, n), np.int32) if pend else None
        na = np.zeros(n, np.float32)
        L.check(self.lib.sim_read_state(
            self.h, net, v.ctypes.data_as(C.POINTER(C.c_float)),
            ca.ctypes.data_as(C.POINTER(C.c_float)), ref.ctypes.data_as(C.POINTER(C.c_uint8)),
            pd.ctypes.data_as(C.POINTER(C.c_int32)) if pend else None,
            na.ctypes.data_as(C.POINTER(C.c_float))), self.h)
        return {"v": v, "ca": ca, "ref": ref, "pend": pd, "na": na, "now": self.now}

    def synapses(self, net: int = 0, i0: int = 0, i1: int | None = None):
        """(row_ptr, tgt, dly, wq) of source rows [i0, i1) in canonical order."""
        if i1 is None:
            i1 = self.net_neurons(net)
        rp = np.zeros(i1 - i0 + 1, np.int64)
        rc = self.lib.sim_read_synapses(self.h, net, i0, i1, rp.ctypes.data_as(C.POINTER(C.c_int64)),
                                        None, None, None, 0)
        if rc not in (L.OK, L.ETRUNC):
            L.check(rc, self.h)
        total = int(rp[-1])
        tgt = np.zeros(max(total, 1), np.int32)
        dly = np.zeros(max(total, 1), np.uint8)
        wq = np.zeros(max(total, 1), np.int16)
        L.check(self.lib.sim_read_synapses(
            self.h, net, i0, i1, rp.ctypes.data_as(C.POINTER(C.c_int64)),
            tgt.ctypes.data_as(C.POINTER(C.c_int32)), dly.ctypes.data_as(C.POINTER(C.c_uint8)),
            wq.ctypes.data_as(C.POINTER(C.c_int16)), total), self.h)
        return rp, tgt[:total], dly[:total], wq[:total]

    # -- state management ---------------------------------------------------------------------
    def save(self, slot: int = 0):
        L.check(self.lib.sim_save(self.h, slot), self.h)

    def restore(self, slot: int = 0):
        L.check(self.lib.sim_restore(self.h, slot), self.h)

    def set_launch(self, delivery: int | None = None, block: int | None = None,
                   tile: tuple[int, int] | None = None, graph_steps: int | None = None,
                   gather_steps: int | None = None):
        """Change the launch configuration; None keeps the current value."""
        cur = self.get_launch()
        lc = L.SimLaunch()
        lc.delivery = cur["delivery"] if delivery is None else int(delivery)
        lc.block = cur["block"] if block is None else int(block)
        tx, ty = cur["tile"] if tile is None else tile
        lc.tile_x, lc.tile_y = int(tx), int(ty)
        lc.graph_steps = cur["graph_steps"] if graph_steps is None else int(graph_steps)
        if gather_steps is None:  # keep the window, unless the tile changes: then automatic
            gather_steps = cur["gather_steps"] if tile is None else 0
        lc.gather_steps = int(gather_steps)
        L.check(self.lib.sim_set_launch(self.h, C.byref(lc)), self.h)

    def get_launch(self) -> dict:
        lc = L.SimLaunch()
        L.check(self.lib.sim_get_launch(self.h, C.byref(lc)), self.h)
        return {"delivery": lc.delivery, "block": lc.block, "tile": (lc.tile_x, lc.tile_y),
                "graph_steps": lc.graph_steps, "gather_steps": lc.gather_steps}

    def digest(self) -> int:
        d = C.c_uint64()
        L.check(self.lib.sim_state_digest(self.h, C.byref(d)), self.h)
        return d.value

    def autotune(self, window: int = 20, cache_path: str | None = None) -> dict:
        """Measure the candidate launch configurations from the current state and keep the
        fastest (the state is restored afterwards)."""
        lc = L.SimLaunch()
        ms = C.c_double()
        L.check(self.lib.sim_autotune(self.h, int(window),
                                      cache_path.encode() if cache_path else None,
                                      C.byref(lc), C.byref(ms)), self.h)
        return {"delivery": lc.delivery, "block": lc.block, "tile": (lc.tile_x, lc.tile_y),
                "graph_steps": lc.graph_steps, "gather_steps": lc.gather_steps,
                "ms_per_step": ms.value}

    def set_params(self, tau_m: float, g_ahp: float):
        L.check(self.lib.sim_set_params(self.h, float(tau_m), float(g_ahp)), self.h)

    def set_timing(self, on: bool = True):
        L.check(self.lib.sim_set_timing(self.h, 1 if on else 0), self.h)

    def timing(self) -> dict:
        """Per-kernel-class totals of the last step() call (timing must be on)."""
        ms = (C.c_double * 6)()
        L.check(self.lib.sim_get_timing(self.h, ms, 6), self.h)
        names = ("update", "deliver", "raster")
        return {names[c]: {"ms": ms[c], "launches": int(ms[3 + c])} for c in range(3)}

    # -- train mode ---------------------------------------------------------------------------
    @staticmethod
    def _dev(t, dtype_name: str, n: int):
        import torch
        if not (t.is_cuda and t.is_contiguous() and t.dtype == getattr(torch, dtype_name)
                and t.numel() == n):
            raise ValueError(f"expected a contiguous device {dtype_name} tensor of {n} elements")
        return C.c_void_p(t.data_ptr())

    def rewind(self):
        L.check(self.lib.sim_rewind(self.h), self.h)

    def set_weights(self, w):
        """Master weights (device float32 [n_synapses], mV, canonical order)."""
        L.check(self.lib.sim_set_weights(self.h, self._dev(w, "float32", self.n_synapses)), self.h)

    def get_weights(self):
        import torch
        w = torch.empty(self.n_synapses, dtype=torch.float32, device="cuda")
        L.check(self.lib.sim_get_weights(self.h, self._dev(w, "float32", self.n_synapses)), self.h)
        return w

    def column_rates(self):
        """Mean rate of every column since step 0 (Hz), device float32 [n_cols]."""
        import torch
        r = torch.empty(self.n_cols, dtype=torch.float32, device="cuda")
        L.check(self.lib.sim_column_rates(self.h, self._dev(r, "float32", self.n_cols)), self.h)
        return r

    def backward(self, grad_rates):
        """Surrogate-gradient backward through [0, now) for a given dL/dR (sim_backward_rates):
        returns (dL/dw as device float32 [n_synapses] in canonical order, dL/dtau_m,
        dL/dg_AHP)."""
        import torch
        gr = grad_rates.detach().to(torch.float32).contiguous()
        gw = torch.empty(self.n_synapses, dtype=torch.float32, device="cuda")
        gt, gg = C.c_double(), C.c_double()
        L.check(self.lib.sim_backward_rates(self.h, self._dev(gr, "float32", self.n_cols),
                                            self._dev(gw, "float32", self.n_synapses),
                                            C.byref(gt), C.byref(gg)), self.h)
        return gw, gt.value, gg.value

    def backward_loss(self, target_rates):
        """sim_backward: the built-in loss L = mean_c (R_c - R*_c)^2 of the column rates since
        step 0 against the targets; returns (L, dL/dw, dL/dtau_m, dL/dg_AHP)."""
        import torch
        tg = torch.as_tensor(target_rates, dtype=torch.float32, device="cuda").contiguous()
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        gw = torch.empty(self.n_synapses, dtype=torch.float32, device="cuda")
        gt, gg = C.c_double(), C.c_double()
        L.check(self.lib.sim_backward(self.h, self._dev(tg, "float32", self.n_cols),
                                      self._dev(loss, "float32", 1),
                                      self._dev(gw, "float32", self.n_synapses), C.byref(gt),
                                      C.byref(gg)), self.h)
        return float(loss.item()), gw, gt.value, gg.value


def _column_rates_fn():
    import torch

    class ColumnRates(torch.autograd.Function):
        """rates = simulate(w, tau_m, g_AHP) over `steps` steps from the initial state;
        the backward is the library's surrogate-gradient adjoint."""

        @staticmethod
        def forward(ctx, w, tau_m, g_ahp, sim, steps):
            ctx.devs = tuple(x.device if torch.is_tensor(x) else None for x in (tau_m, g_ahp))
            sim.rewind()
            sim.set_params(float(tau_m), float(g_ahp))
            sim.set_weights(w.detach().contiguous())
            sim.step(int(steps))
            ctx.sim = sim
            return sim.column_rates()

        @staticmethod
        def backward(ctx, grad_rates):
            gw, gt, gg = ctx.sim.backward(grad_rates)
            scal = [None if d is None else torch.tensor(v, dtype=torch.float64, device=d)
                    for v, d in zip((gt, gg), ctx.devs)]
            return gw, scal[0], scal[1], None, None

    return ColumnRates


def column_rates(sim: Simulation, w, tau_m, g_ahp, steps: int):
    """Differentiable mean column rates of a train-mode Simulation (see ColumnRates)."""
    return _column_rates_fn().apply(w, tau_m, g_ahp, sim, steps)
