"""ctypes binding of libdpsnn.so (argument marshalling only; include/dpsnn.h is the contract).

Loading fails loudly if the library was not built: there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpsnn.so")

OK, EINVAL, ENOMEM, EHIP, ESTATE, ETRUNC = 0, -1, -2, -3, -4, -5
DELIVERY_AUTO, DELIVERY_ARRIVAL, DELIVERY_PUSH = 0, 1, 2
NEURON_LIF, NEURON_IZHIKEVICH = 0, 1
CONN_EXP3X3, CONN_GAUSS = 0, 1

#: Every entry point declared in include/dpsnn.h.
EXPORTS = [
    "sim_create", "sim_destroy", "sim_step", "sim_sync", "sim_read_spikes", "sim_backward",
    "sim_last_error", "sim_get_info", "sim_get_stats", "sim_now", "sim_read_state",
    "sim_read_synapses", "sim_save", "sim_restore", "sim_set_weights", "sim_get_weights",
    "sim_set_params", "sim_get_launch", "sim_set_launch", "sim_set_timing", "sim_get_timing",
    "sim_state_digest", "sim_autotune", "sim_rewind", "sim_column_rates",
    "sim_read_spikes_static", "sim_query_sizes", "sim_backward_rates", "sim_tune_tiling",
]


class SimNet(C.Structure):
    _fields_ = [("rows", C.c_int32), ("cols", C.c_int32), ("seed", C.c_uint64),
                ("ext_rate_hz", C.c_double)]


class SimConfig(C.Structure):
    _fields_ = [
        ("npc", C.c_int32), ("n_exc", C.c_int32),
        ("p_own", C.c_double), ("p_remote", C.c_double), ("decay_um", C.c_double),
        ("spacing_um", C.c_double),
        ("d_min", C.c_int32), ("d_max", C.c_int32),
        ("we_mu", C.c_double), ("we_sigma", C.c_double), ("wi_mu", C.c_double),
        ("wi_sigma", C.c_double),
        ("tau_m", C.c_double), ("theta", C.c_double), ("v_reset", C.c_double),
        ("t_ref", C.c_int32),
        ("tau_ca", C.c_double), ("ca_inc", C.c_double), ("g_ahp", C.c_double), ("dt", C.c_double),
        ("ext_syn", C.c_int32), ("j_ext", C.c_double),
        ("n_nets", C.c_int32), ("nets", C.POINTER(SimNet)),
        ("delivery", C.c_int32), ("block", C.c_int32),
        ("tile_x", C.c_int32), ("tile_y", C.c_int32),
        ("record_steps", C.c_int64), ("raster_capacity", C.c_int64),
        ("train_mode", C.c_int32), ("ckpt_every", C.c_int32),
        ("surrogate_beta", C.c_double),
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


class SimLaunch(C.Structure):
    _fields_ = [("delivery", C.c_int32), ("block", C.c_int32), ("tile_x", C.c_int32),
                ("tile_y", C.c_int32), ("graph_steps", C.c_int32),
                ("gather_steps", C.c_int32)]


class SimInfo(C.Structure):
    _fields_ = [("n_nets", C.c_int32), ("n_cols", C.c_int32), ("n_neurons", C.c_int64),
                ("n_synapses", C.c_int64), ("ring_slots", C.c_int32),
                ("device_bytes", C.c_int64), ("caller_bytes", C.c_int64)]


class SimSizes(C.Structure):
    _fields_ = [("n_neurons", C.c_int64), ("n_records", C.c_int64),
                ("synapse_bytes", C.c_uint64), ("index_bytes", C.c_uint64),
                ("state_bytes", C.c_uint64), ("history_bytes", C.c_uint64),
                ("state_v_offset", C.c_uint64), ("state_ca_offset", C.c_uint64),
                ("state_ref_offset", C.c_uint64)]


class SimBuffers(C.Structure):
    _fields_ = [("synapses", C.c_void_p), ("synapse_bytes", C.c_uint64),
                ("index", C.c_void_p), ("index_bytes", C.c_uint64),
                ("state", C.c_void_p), ("state_bytes", C.c_uint64),
                ("history", C.c_void_p), ("history_bytes", C.c_uint64)]

#: The four caller-ownable regions: (SimBuffers pointer field, size field, SimSizes field).
REGIONS = (("synapses", "synapse_bytes"), ("index", "index_bytes"), ("state", "state_bytes"),
           ("history", "history_bytes"))


class SimStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("spikes", C.c_int64), ("events_recurrent", C.c_int64),
                ("events_external", C.c_int64), ("synapses_streamed", C.c_int64),
                ("synapses_delivered", C.c_int64)]


_lib = None


def lib():
    """Load libdpsnn.so; raises if it is missing (build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libdpsnn.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp = C.c_void_p
    sigs = {
        "sim_query_sizes": (C.c_int, [P(SimConfig), P(SimSizes)]),
        "sim_create": (C.c_int, [P(SimConfig), P(SimBuffers), vp, P(vp)]),
        "sim_destroy": (None, [vp]),
        "sim_step": (C.c_int, [vp, C.c_int64]),
        "sim_sync": (C.c_int, [vp]),
        "sim_read_spikes": (C.c_int, [vp, C.c_int32, C.c_int64, C.c_int64, P(C.c_int64),
                                      P(C.c_int32), C.c_int64, P(C.c_int64)]),
        "sim_read_spikes_static": (C.c_int, [vp, C.c_int32, C.c_int64, C.c_int64,
                                             P(C.c_int64), P(C.c_int32), C.c_int64,
                                             P(C.c_int64)]),
        "sim_backward": (C.c_int, [vp, vp, vp, vp, P(C.c_double), P(C.c_double)]),
        "sim_backward_rates": (C.c_int, [vp, vp, vp, P(C.c_double), P(C.c_double)]),
        "sim_last_error": (C.c_char_p, [vp]),
        "sim_get_info": (C.c_int, [vp, P(SimInfo)]),
        "sim_get_stats": (C.c_int, [vp, C.c_int32, P(SimStats)]),
        "sim_now": (C.c_int64, [vp]),
        "sim_read_state": (C.c_int, [vp, C.c_int32, P(C.c_float), P(C.c_float), P(C.c_uint8),
                                     P(C.c_int32), P(C.c_float)]),
        "sim_read_synapses": (C.c_int, [vp, C.c_int32, C.c_int64, C.c_int64, P(C.c_int64),
                                        P(C.c_int32), P(C.c_uint8), P(C.c_int16), C.c_int64]),
        "sim_save": (C.c_int, [vp, C.c_int32]),
        "sim_restore": (C.c_int, [vp, C.c_int32]),
        "sim_set_weights": (C.c_int, [vp, vp]),
        "sim_get_weights": (C.c_int, [vp, vp]),
        "sim_set_params": (C.c_int, [vp, C.c_double, C.c_double]),
        "sim_get_launch": (C.c_int, [vp, P(SimLaunch)]),
        "sim_set_launch": (C.c_int, [vp, P(SimLaunch)]),
        "sim_set_timing": (C.c_int, [vp, C.c_int32]),
        "sim_get_timing": (C.c_int, [vp, P(C.c_double), C.c_int32]),
        "sim_state_digest": (C.c_int, [vp, P(C.c_uint64)]),
        "sim_autotune": (C.c_int, [vp, C.c_int32, C.c_char_p, P(SimLaunch), P(C.c_double)]),
        "sim_tune_tiling": (C.c_int, [P(SimConfig), C.c_int32, C.c_int32, P(C.c_int32),
                                      P(C.c_int32), P(C.c_double)]),
        "sim_rewind": (C.c_int, [vp]),
        "sim_column_rates": (C.c_int, [vp, vp]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


class DpsnnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("dpsnn error %d: %s" % (code, msg))
        self.code = code


def check(rc: int, handle=None):
    if rc != OK:
        msg = lib().sim_last_error(handle)
        raise DpsnnError(rc, msg.decode() if msg else "")
    return rc
