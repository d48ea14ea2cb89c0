"""CPU oracle of the DPSNN per-1 ms simulation step -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  The product path (the HIP library and its Python binding) never
does, and this package never imports the product package.  The shared inputs are plain
parameter dictionaries (see ``paper_1511_09325_amd.workloads``), which hold no arithmetic
of the method.

This module is a thin ctypes binding of ``dpsnn_oracle.c`` (built with gcc by
:func:`build`), plus the FP64 adjoint of ``dpsnn_adjoint.c``.  Each C function cites the
paper passage it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libdpsnn_oracle.so")
_SOURCES = ["dpsnn_oracle.c", "dpsnn_adjoint.c"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no fast-math, no FP contraction."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", tmp] + srcs + ["-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _SO)
    return _SO


class _Cfg(C.Structure):
    _fields_ = [
        ("rows", C.c_int32), ("cols", C.c_int32), ("npc", C.c_int32), ("n_exc", C.c_int32),
        ("seed", C.c_uint64),
        ("p_own", C.c_double), ("p_remote", C.c_double), ("decay_um", C.c_double),
        ("spacing_um", C.c_double),
        ("d_min", C.c_int32), ("d_max", C.c_int32),
        ("we_mu", C.c_double), ("we_sigma", C.c_double), ("wi_mu", C.c_double),
        ("wi_sigma", C.c_double),
        ("tau_m", C.c_double), ("theta", C.c_double), ("v_reset", C.c_double),
        ("t_ref", C.c_int32),
        ("tau_ca", C.c_double), ("ca_inc", C.c_double), ("g_ahp", C.c_double), ("dt", C.c_double),
        ("ext_rate_hz", C.c_double), ("ext_syn", C.c_int32), ("j_ext", C.c_double),
        ("neuron_model", C.c_int32), ("tau_na", C.c_double), ("na_inc", C.c_double),
        ("g_na", C.c_double),
        ("izh_a_e", C.c_double), ("izh_b_e", C.c_double), ("izh_c_e", C.c_double),
        ("izh_d_e", C.c_double),
        ("izh_a_i", C.c_double), ("izh_b_i", C.c_double), ("izh_c_i", C.c_double),
        ("izh_d_i", C.c_double), ("izh_vpeak", C.c_double),
        ("conn_kernel", C.c_int32), ("lateral_amp", C.c_double),
        ("lateral_sigma_um", C.c_double), ("lateral_cutoff", C.c_double),
        ("stdp", C.c_int32), ("stdp_tau_plus", C.c_double), ("stdp_tau_minus", C.c_double),
        ("stdp_a_plus", C.c_double), ("stdp_a_minus", C.c_double), ("stdp_w_max", C.c_double),
    ]

NEURON_LIF, NEURON_IZHIKEVICH = 0, 1
CONN_EXP3X3, CONN_GAUSS = 0, 1


class _AdjParams(C.Structure):
    _fields_ = [("pm", C.c_double), ("pc", C.c_double), ("gamma", C.c_double),
                ("alpha", C.c_double), ("theta", C.c_double), ("vreset", C.c_double),
                ("beta", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = C.CDLL(_SO)
        P = C.POINTER
        u32p, i32p, i64p, u8p, i16p, f32p, f64p, u64p = (
            P(C.c_uint32), P(C.c_int32), P(C.c_int64), P(C.c_uint8), P(C.c_int16), P(C.c_float),
            P(C.c_double), P(C.c_uint64))
        cp = P(_Cfg)
        sig = {
            "orc_set_threads": (None, [C.c_int32]),
            "orc_stencil_radius": (C.c_int32, [cp]),
            "orc_threads": (C.c_int32, []),
            "orc_philox": (None, [u32p, u32p, u32p]),
            "orc_column_probability": (C.c_double, [cp, C.c_int32, C.c_int32]),
            "orc_pair": (C.c_int, [cp, C.c_int64, C.c_int64, i32p, i16p]),
            "orc_row": (C.c_int64, [cp, C.c_int64, i32p, u8p, i16p, C.c_int64]),
            "orc_network": (C.c_int64, [cp, i64p, i32p, u8p, i16p, C.c_int64]),
            "orc_poisson_table": (None, [C.c_double, u64p]),
            "orc_poisson_count": (C.c_int32, [u64p, C.c_uint32]),
            "orc_initial_v": (C.c_float, [cp, C.c_int64]),
            "orc_initial_state": (None, [cp, C.c_int64, f32p, f32p]),
            "orc_sim_get_na": (None, [C.c_void_p, f32p]),
            "orc_sim_get_weights": (None, [C.c_void_p, i16p]),
            "orc_stdp_synapse": (C.c_int16, [cp, C.c_int64, u8p, u8p, C.c_int32, C.c_int16]),
            "orc_sim_set_na": (None, [C.c_void_p, f32p]),
            "orc_ext_counts": (None, [cp, C.c_int64, C.c_int64, C.c_int64, i32p]),
            "orc_neuron_update": (C.c_int, [cp, C.c_int64, C.c_int64, C.c_int32, f32p, f32p, u8p,
                                            f32p]),
            "orc_update_many": (None, [cp, C.c_int64, C.c_int64, C.c_int64, i32p, f32p, f32p,
                                       u8p, u8p, f32p]),
            "orc_input_brute": (None, [cp, C.c_int64, i64p, C.c_int64, C.c_int64, u8p,
                                       C.c_int64, C.c_int64, i32p]),
            "orc_sim_consumed": (C.c_int64, [C.c_void_p]),
            "orc_sim_create": (C.c_void_p, [cp, C.c_int64, i64p, i32p, u8p, i32p]),
            "orc_sim_destroy": (None, [C.c_void_p]),
            "orc_sim_step": (C.c_int, [C.c_void_p, C.c_int64]),
            "orc_sim_now": (C.c_int64, [C.c_void_p]),
            "orc_sim_ring_slots": (C.c_int32, [C.c_void_p]),
            "orc_sim_spikes": (C.c_int64, [C.c_void_p, C.c_int64, i32p, C.c_int64]),
            "orc_sim_counts": (None, [C.c_void_p, i64p, i64p, i64p]),
            "orc_sim_get_state": (None, [C.c_void_p, f32p, f32p, u8p, i32p]),
            "orc_sim_set_state": (None, [C.c_void_p, C.c_int64, f32p, f32p, u8p, i32p]),
            "orc_sim_inject": (None, [C.c_void_p, C.c_int32, C.c_int64, C.c_int32]),
            "orc_sim_record": (None, [C.c_void_p, C.c_int]),
            "orc_sim_trajectory": (C.c_int64, [C.c_void_p, f32p, f32p, f32p, u8p, u8p, i32p,
                                               C.c_int64]),
        }
        ap = P(_AdjParams)
        sig["orc_adjoint"] = (C.c_int, [
            ap, C.c_int64, C.c_int64, i64p, i32p, u8p, f64p,   # params, n, T, csr, w (mV)
            f64p, f64p, f64p, f64p, u8p,                        # v_prev, ca_prev, v_tilde, s, r
            f64p, f64p, f64p, f64p, f64p])                      # dL/ds, dL/dV~, grad_w, grad_pm,
                                                                # grad_gamma
        sig["orc_soft_forward"] = (C.c_int, [
            cp, ap, C.c_int64, C.c_int64, i64p, i32p, u8p, f64p, f64p, f64p, f64p, f64p])
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Host threads of the oracle's loops over independent rows and neurons (results do not
    depend on it)."""
    lib().orc_set_threads(int(n))


def threads() -> int:
    return int(lib().orc_threads())


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def make_config(p: dict) -> _Cfg:
    c = _Cfg()
    for name, ctype in _Cfg._fields_:
        setattr(c, name, ctype(p[name]).value)
    return c


# ---------------------------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------------------------
def philox(ctr, key):
    """Philox4x32-10 block function (Salmon et al., SC'11)."""
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def column_probability(p: dict, src_col: int, tgt_col: int) -> float:
    cfg = make_config(p)
    return lib().orc_column_probability(C.byref(cfg), src_col, tgt_col)


def pair(p: dict, i: int, j: int):
    cfg = make_config(p)
    d = C.c_int32(0)
    w = C.c_int16(0)
    ok = lib().orc_pair(C.byref(cfg), i, j, C.byref(d), C.byref(w))
    return (bool(ok), d.value, w.value)


def n_neurons(p: dict) -> int:
    return p["rows"] * p["cols"] * p["npc"]


def stencil_radius(p: dict) -> int:
    return int(lib().orc_stencil_radius(C.byref(make_config(p))))


def row(p: dict, i: int):
    cfg = make_config(p)
    cap = 49 * p["npc"] + 1
    tgt = np.zeros(cap, np.int32)
    dly = np.zeros(cap, np.uint8)
    wq = np.zeros(cap, np.int16)
    n = lib().orc_row(C.byref(cfg), i, _ptr(tgt, C.c_int32), _ptr(dly, C.c_uint8),
                      _ptr(wq, C.c_int16), cap)
    assert n >= 0
    return tgt[:n].copy(), dly[:n].copy(), wq[:n].copy()


def network(p: dict):
    """Whole network as CSR: (row_ptr int64[n+1], tgt int32, dly uint8, wq int16 at 2^-14 mV)."""
    cfg = make_config(p)
    n = n_neurons(p)
    cap = n * (9 * p["npc"]) + 1
    cap = min(cap, n * 2 * p["npc"] + 1024)
    row_ptr = np.zeros(n + 1, np.int64)
    tgt = np.zeros(cap, np.int32)
    dly = np.zeros(cap, np.uint8)
    wq = np.zeros(cap, np.int16)
    s = lib().orc_network(C.byref(cfg), _ptr(row_ptr, C.c_int64), _ptr(tgt, C.c_int32),
                          _ptr(dly, C.c_uint8), _ptr(wq, C.c_int16), cap)
    if s < 0:
        raise RuntimeError("oracle network capacity exceeded")
    return row_ptr, tgt[:s].copy(), dly[:s].copy(), wq[:s].copy()


def poisson_table(lam: float):
    tab = np.zeros(63, np.uint64)
    lib().orc_poisson_table(float(lam), _ptr(tab, C.c_uint64))
    return tab


def poisson_count(tab, x: int) -> int:
    t = np.ascontiguousarray(tab, dtype=np.uint64)
    return lib().orc_poisson_count(_ptr(t, C.c_uint64), x)


def ext_counts(p: dict, u: int, j0: int = 0, n: int | None = None):
    """External Poisson counts n_j(u) for neurons j0 .. j0+n-1 at step u."""
    cfg = make_config(p)
    if n is None:
        n = n_neurons(p) - j0
    out = np.zeros(n, np.int32)
    lib().orc_ext_counts(C.byref(cfg), u, j0, n, _ptr(out, C.c_int32))
    return out


def neuron_update(p: dict, j: int, u: int, rec_input: int, v: float, ca: float, ref: int,
                  na: float = 0.0):
    """One neuron's step from its state; returns (spike, v, ca, ref, na)."""
    cfg = make_config(p)
    vv, cc, rr, nn = C.c_float(v), C.c_float(ca), C.c_uint8(ref), C.c_float(na)
    s = lib().orc_neuron_update(C.byref(cfg), j, u, int(rec_input), C.byref(vv), C.byref(cc),
                                C.byref(rr), C.byref(nn))
    return (bool(s), np.float32(vv.value), np.float32(cc.value), int(rr.value),
            np.float32(nn.value))


def stdp_synapse(p: dict, pre, post, d: int, q0: int) -> int:
    """The plasticity rule on one synapse (delay d, weight q0 at step 0) from its source's and
    its target's spike flags over steps 0 .. T-1: its weight after step T-1."""
    pre = np.ascontiguousarray(pre, np.uint8)
    post = np.ascontiguousarray(post, np.uint8)
    assert pre.shape == post.shape
    return int(lib().orc_stdp_synapse(C.byref(make_config(p)), len(pre), _ptr(pre, C.c_uint8),
                                      _ptr(post, C.c_uint8), int(d), int(q0)))


def update_many(p: dict, u: int, rec_input, v, ca, ref, j0: int = 0, na=None):
    """neuron_update for neurons j0 .. j0+n-1 at step u on copies of the given state;
    returns (spike flags, v, ca, ref) and, when na is given, the new na as a fifth item."""
    cfg = make_config(p)
    ri = np.ascontiguousarray(rec_input, np.int32)
    v2 = np.array(v, np.float32)
    c2 = np.array(ca, np.float32)
    r2 = np.array(ref, np.uint8)
    n2 = None if na is None else np.array(na, np.float32)
    spk = np.zeros(len(ri), np.uint8)
    lib().orc_update_many(C.byref(cfg), u, j0, len(ri), _ptr(ri, C.c_int32),
                          _ptr(v2, C.c_float), _ptr(c2, C.c_float), _ptr(r2, C.c_uint8),
                          _ptr(spk, C.c_uint8), None if n2 is None else _ptr(n2, C.c_float))
    return (spk, v2, c2, r2) if n2 is None else (spk, v2, c2, r2, n2)


def input_brute(p: dict, targets, t_arr: int, t_emit_max: int, mask, mask_t0: int):
    """Recurrent input arriving at step t_arr at each target, summed over every synapse
    (decided again pair by pair) whose source spiked at an emission step <= t_emit_max;
    mask[e - mask_t0][i] marks the spikes of step e."""
    cfg = make_config(p)
    t = np.ascontiguousarray(targets, np.int64)
    m = np.ascontiguousarray(mask, np.uint8)
    assert m.ndim == 2 and m.shape[1] == n_neurons(p)
    out = np.zeros(len(t), np.int32)
    lib().orc_input_brute(C.byref(cfg), len(t), _ptr(t, C.c_int64), t_arr, t_emit_max,
                          _ptr(m, C.c_uint8), mask_t0, m.shape[0], _ptr(out, C.c_int32))
    return out


def initial_v(p: dict, j: int) -> float:
    cfg = make_config(p)
    return lib().orc_initial_v(C.byref(cfg), j)


def initial_state(p: dict, j: int):
    """(v, ca) of neuron j at step 0 (ca: the Izhikevich recovery variable for that model)."""
    cfg = make_config(p)
    v, ca = C.c_float(), C.c_float()
    lib().orc_initial_state(C.byref(cfg), j, C.byref(v), C.byref(ca))
    return np.float32(v.value), np.float32(ca.value)


# ---------------------------------------------------------------------------------------------
# simulation
# ---------------------------------------------------------------------------------------------
class Sim:
    """Plain push-form simulation: ring[D][n] of int32 input, D = d_max + 1."""

    def __init__(self, p: dict, net=None, w32=None):
        """net: (row_ptr, tgt, dly, wq) CSR; built from p if None.  w32 overrides the
        2^-16 mV efficacies (default 4 * wq)."""
        self.p = dict(p)
        self._cfg = make_config(p)
        if net is None:
            net = network(p)
        row_ptr, tgt, dly, wq = net
        self.row_ptr = np.ascontiguousarray(row_ptr, np.int64)
        self.tgt = np.ascontiguousarray(tgt, np.int32)
        self.dly = np.ascontiguousarray(dly, np.uint8)
        if w32 is None:
            w32 = np.asarray(wq, np.int32) * 4
        self.w32 = np.ascontiguousarray(w32, np.int32)
        self.n = len(self.row_ptr) - 1
        L = lib()
        self._h = L.orc_sim_create(C.byref(self._cfg), self.n, _ptr(self.row_ptr, C.c_int64),
                                   _ptr(self.tgt, C.c_int32), _ptr(self.dly, C.c_uint8),
                                   _ptr(self.w32, C.c_int32))
        self.D = L.orc_sim_ring_slots(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_sim_destroy(h)
            self._h = None

    @property
    def now(self) -> int:
        return lib().orc_sim_now(self._h)

    def step(self, n: int = 1):
        lib().orc_sim_step(self._h, n)

    def spikes(self, u: int):
        cap = self.n
        ids = np.zeros(max(cap, 1), np.int32)
        k = lib().orc_sim_spikes(self._h, u, _ptr(ids, C.c_int32), cap)
        return ids[:k].copy()

    def raster(self, t0: int, t1: int):
        return [self.spikes(u) for u in range(t0, t1)]

    def counts(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        lib().orc_sim_counts(self._h, C.byref(a), C.byref(b), C.byref(c))
        return {"spikes": a.value, "e_rec": b.value, "e_ext": c.value}

    def consumed(self) -> int:
        return lib().orc_sim_consumed(self._h)

    def state(self):
        v = np.zeros(self.n, np.float32)
        ca = np.zeros(self.n, np.float32)
        ref = np.zeros(self.n, np.uint8)
        pend = np.zeros((self.D, self.n), np.int32)
        lib().orc_sim_get_state(self._h, _ptr(v, C.c_float), _ptr(ca, C.c_float),
                                _ptr(ref, C.c_uint8), _ptr(pend, C.c_int32))
        na = np.zeros(self.n, np.float32)
        lib().orc_sim_get_na(self._h, _ptr(na, C.c_float))
        return {"v": v, "ca": ca, "ref": ref, "pend": pend, "na": na, "now": self.now}

    def set_state(self, now, v, ca, ref, pend, na=None):
        v = np.ascontiguousarray(v, np.float32)
        ca = np.ascontiguousarray(ca, np.float32)
        ref = np.ascontiguousarray(ref, np.uint8)
        pend = np.ascontiguousarray(pend, np.int32)
        assert pend.shape == (self.D, self.n)
        lib().orc_sim_set_state(self._h, now, _ptr(v, C.c_float), _ptr(ca, C.c_float),
                                _ptr(ref, C.c_uint8), _ptr(pend, C.c_int32))
        if na is not None:
            na = np.ascontiguousarray(na, np.float32)
            lib().orc_sim_set_na(self._h, _ptr(na, C.c_float))

    def weights(self):
        """Current weights (int16, 2^-14 mV) in CSR order (plasticity changes them)."""
        wq = np.zeros(max(len(self.tgt), 1), np.int16)
        lib().orc_sim_get_weights(self._h, _ptr(wq, C.c_int16))
        return wq[:len(self.tgt)]

    def inject(self, q: int, j: int, value: int):
        lib().orc_sim_inject(self._h, q, j, value)

    def record(self, on: bool = True):
        lib().orc_sim_record(self._h, 1 if on else 0)

    def trajectory(self, steps: int):
        shape = (steps, self.n)
        vp = np.zeros(shape, np.float32)
        cp = np.zeros(shape, np.float32)
        vt = np.zeros(shape, np.float32)
        s = np.zeros(shape, np.uint8)
        r = np.zeros(shape, np.uint8)
        a = np.zeros(shape, np.int32)
        m = lib().orc_sim_trajectory(self._h, _ptr(vp, C.c_float), _ptr(cp, C.c_float),
                                     _ptr(vt, C.c_float), _ptr(s, C.c_uint8), _ptr(r, C.c_uint8),
                                     _ptr(a, C.c_int32), steps)
        return {"v_prev": vp[:m], "ca_prev": cp[:m], "v_tilde": vt[:m], "s": s[:m], "r": r[:m],
                "input": a[:m]}


# ---------------------------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------------------------
def step_constants(p: dict, single: bool):
    """Step constants; single=True gives the float32-rounded values the hard step uses."""
    pm = np.exp(-p["dt"] / p["tau_m"])
    pc = np.exp(-p["dt"] / p["tau_ca"])
    gam = p["g_ahp"] * p["dt"]
    vals = dict(pm=pm, pc=pc, gamma=gam, alpha=p["ca_inc"], theta=p["theta"], vreset=p["v_reset"])
    if single:
        vals = {k: float(np.float32(v)) for k, v in vals.items()}
    return vals


def _adj_params(consts: dict, beta: float):
    a = _AdjParams()
    for k, v in consts.items():
        setattr(a, k, float(v))
    a.beta = float(beta)
    return a


def adjoint(consts: dict, beta: float, net, w_mv, traj: dict, dl_ds, dl_dvt=None):
    """FP64 reverse recursion over a trajectory; returns (grad_w, grad_pm, grad_gamma).
    dl_dvt: optional direct dL/dV~ ([T][n])."""
    row_ptr, tgt, dly = (np.ascontiguousarray(net[0], np.int64),
                         np.ascontiguousarray(net[1], np.int32),
                         np.ascontiguousarray(net[2], np.uint8))
    n = len(row_ptr) - 1
    T = traj["v_tilde"].shape[0]
    f = lambda a: np.ascontiguousarray(a, np.float64)
    vp, cp, vt, s = f(traj["v_prev"]), f(traj["ca_prev"]), f(traj["v_tilde"]), f(traj["s"])
    r = np.ascontiguousarray(traj.get("r", np.zeros((T, n), np.uint8)), np.uint8)
    w = f(w_mv)
    dl = f(dl_ds)
    dv = None if dl_dvt is None else f(dl_dvt)
    gw = np.zeros(len(tgt), np.float64)
    gpm, ggam = C.c_double(), C.c_double()
    k = _adj_params(consts, beta)
    rc = lib().orc_adjoint(C.byref(k), n, T, _ptr(row_ptr, C.c_int64), _ptr(tgt, C.c_int32),
                           _ptr(dly, C.c_uint8), _ptr(w, C.c_double), _ptr(vp, C.c_double),
                           _ptr(cp, C.c_double), _ptr(vt, C.c_double), _ptr(s, C.c_double),
                           _ptr(r, C.c_uint8), _ptr(dl, C.c_double),
                           None if dv is None else _ptr(dv, C.c_double), _ptr(gw, C.c_double),
                           C.byref(gpm), C.byref(ggam))
    assert rc == 0
    return gw, gpm.value, ggam.value


def soft_forward(p: dict, consts: dict, beta: float, net, w_mv, T: int):
    """FP64 soft-spike forward; returns the trajectory dict ([T][n] arrays)."""
    cfg = make_config(p)
    row_ptr, tgt, dly = (np.ascontiguousarray(net[0], np.int64),
                         np.ascontiguousarray(net[1], np.int32),
                         np.ascontiguousarray(net[2], np.uint8))
    n = len(row_ptr) - 1
    w = np.ascontiguousarray(w_mv, np.float64)
    out = {k: np.zeros((T, n), np.float64) for k in ("v_prev", "ca_prev", "v_tilde", "s")}
    k = _adj_params(consts, beta)
    rc = lib().orc_soft_forward(C.byref(cfg), C.byref(k), n, T, _ptr(row_ptr, C.c_int64),
                                _ptr(tgt, C.c_int32), _ptr(dly, C.c_uint8), _ptr(w, C.c_double),
                                _ptr(out["v_prev"], C.c_double), _ptr(out["ca_prev"], C.c_double),
                                _ptr(out["v_tilde"], C.c_double), _ptr(out["s"], C.c_double))
    assert rc == 0
    return out
