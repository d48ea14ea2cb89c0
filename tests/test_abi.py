"""The C ABI library without a GPU: it loads, exports every entry point that
include/dpsnn.h declares, the ctypes mirror of its structs matches the C layout, and
configuration errors are rejected before any device work."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_1511_09325_amd import _lib as L
from paper_1511_09325_amd import workloads as W
from paper_1511_09325_amd.sim import make_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpsnn.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sim_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libdpsnn.so is not built; run __graft_entry__.build()")
    return L.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 20
    assert sorted(names) == sorted(L.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_error_codes_match_header():
    text = open(HEADER).read()
    codes = dict(re.findall(r"#define (DPSNN_E[A-Z]+) \((-\d+)\)", text))
    assert int(codes["DPSNN_EINVAL"]) == L.EINVAL
    assert int(codes["DPSNN_ENOMEM"]) == L.ENOMEM
    assert int(codes["DPSNN_EHIP"]) == L.EHIP
    assert int(codes["DPSNN_ESTATE"]) == L.ESTATE
    assert int(codes["DPSNN_ETRUNC"]) == L.ETRUNC


_PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "dpsnn.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m));
int main(void) {
  printf("sim_config_t %zu\nsim_net_t %zu\nsim_info_t %zu\nsim_stats_t %zu\n",
         sizeof(sim_config_t), sizeof(sim_net_t), sizeof(sim_info_t), sizeof(sim_stats_t));
  printf("sim_sizes_t %zu\nsim_buffers_t %zu\n", sizeof(sim_sizes_t), sizeof(sim_buffers_t));
  F(sim_config_t, nets) F(sim_config_t, delivery) F(sim_config_t, record_steps)
  F(sim_config_t, ckpt_every) F(sim_config_t, j_ext) F(sim_net_t, ext_rate_hz)
  F(sim_config_t, stdp) F(sim_config_t, stdp_w_max)
  F(sim_info_t, device_bytes) F(sim_info_t, caller_bytes)
  F(sim_sizes_t, history_bytes) F(sim_sizes_t, state_ref_offset)
  F(sim_buffers_t, state) F(sim_buffers_t, history_bytes)
  return 0;
}
"""


def test_struct_layout_matches_c():
    with tempfile.TemporaryDirectory() as td:
        src, exe = os.path.join(td, "p.c"), os.path.join(td, "p")
        open(src, "w").write(_PROBE)
        subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), src, "-o", exe])
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    got = dict(line.split() for line in out.strip().splitlines())
    assert int(got["sim_config_t"]) == C.sizeof(L.SimConfig)
    assert int(got["sim_net_t"]) == C.sizeof(L.SimNet)
    assert int(got["sim_info_t"]) == C.sizeof(L.SimInfo)
    assert int(got["sim_stats_t"]) == C.sizeof(L.SimStats)
    assert int(got["sim_sizes_t"]) == C.sizeof(L.SimSizes)
    assert int(got["sim_buffers_t"]) == C.sizeof(L.SimBuffers)
    for key, (cls, field) in {"sim_config_t.nets": (L.SimConfig, "nets"),
                              "sim_info_t.caller_bytes": (L.SimInfo, "caller_bytes"),
                              "sim_sizes_t.history_bytes": (L.SimSizes, "history_bytes"),
                              "sim_sizes_t.state_ref_offset": (L.SimSizes, "state_ref_offset"),
                              "sim_buffers_t.state": (L.SimBuffers, "state"),
                              "sim_buffers_t.history_bytes": (L.SimBuffers, "history_bytes"),
                              "sim_config_t.delivery": (L.SimConfig, "delivery"),
                              "sim_config_t.record_steps": (L.SimConfig, "record_steps"),
                              "sim_config_t.ckpt_every": (L.SimConfig, "ckpt_every"),
                              "sim_config_t.j_ext": (L.SimConfig, "j_ext"),
                              "sim_config_t.stdp": (L.SimConfig, "stdp"),
                              "sim_config_t.stdp_w_max": (L.SimConfig, "stdp_w_max"),
                              "sim_net_t.ext_rate_hz": (L.SimNet, "ext_rate_hz"),
                              "sim_info_t.device_bytes": (L.SimInfo, "device_bytes")}.items():
        assert int(got[key]) == getattr(cls, field).offset, key


@pytest.mark.parametrize("bad", [
    dict(npc=0), dict(npc=5000), dict(n_exc=2000), dict(d_min=0), dict(d_max=40),
    dict(d_min=5, d_max=4), dict(wi_mu=-1.9), dict(tau_m=0.0), dict(t_ref=300),
    dict(p_own=0.9, p_remote=0.4), dict(rows=0), dict(ext_rate_hz=50.0),
    dict(neuron_model=2), dict(g_na=0.1, tau_na=0.0), dict(neuron_model=1, izh_vpeak=float("nan")),
    dict(stdp=1, stdp_tau_plus=0.0), dict(stdp=1, stdp_w_max=2.5), dict(stdp=1, stdp_w_max=0.0),
    dict(stdp=1, stdp_a_minus=-0.01), dict(stdp=1, stdp_a_plus=float("nan")),
    dict(stdp=1, stdp_a_plus=100.0, stdp_tau_plus=1000.0),
])
def test_invalid_configs_are_rejected_before_device_work(lib, bad):
    p = W.grid(2, 2)
    p.update(bad)
    cfg, nets = make_config(p)
    h = C.c_void_p(123)
    rc = lib.sim_create(C.byref(cfg), None, None, C.byref(h))
    assert rc == L.EINVAL
    assert h.value is None
    assert lib.sim_last_error(None)
    sz = L.SimSizes()
    assert lib.sim_query_sizes(C.byref(cfg), C.byref(sz)) == L.EINVAL


@pytest.mark.parametrize("bad", [dict(neuron_model=1), dict(g_na=0.1)])
def test_train_mode_needs_the_one_variable_lif(lib, bad):
    p = W.grid(2, 2)
    p.update(bad)
    cfg, nets = make_config(p, train_mode=True)
    h = C.c_void_p(123)
    assert lib.sim_create(C.byref(cfg), None, None, C.byref(h)) == L.EINVAL
    assert b"train mode" in lib.sim_last_error(None)


@pytest.mark.parametrize("opts,msg", [(dict(train_mode=True), b"train mode"),
                                      (dict(delivery=2), b"arrival form")])
def test_stdp_excludes_train_mode_and_push(lib, opts, msg):
    p = W.grid(2, 2)
    p.update(stdp=1)
    cfg, nets = make_config(p, **opts)
    h = C.c_void_p(123)
    assert lib.sim_create(C.byref(cfg), None, None, C.byref(h)) == L.EINVAL
    assert msg in lib.sim_last_error(None)


def test_tune_tiling_refuses_bad_arguments_before_device_work(lib):
    cfg, nets = make_config(W.grid(2, 2))
    tx, ty, ms = C.c_int32(), C.c_int32(), C.c_double()
    assert lib.sim_tune_tiling(None, 0, 10, C.byref(tx), C.byref(ty), None) == L.EINVAL
    assert lib.sim_tune_tiling(C.byref(cfg), 0, 10, None, C.byref(ty), None) == L.EINVAL
    assert lib.sim_tune_tiling(C.byref(cfg), -1, 10, C.byref(tx), C.byref(ty), None) == L.EINVAL
    assert lib.sim_tune_tiling(C.byref(cfg), 0, 0, C.byref(tx), C.byref(ty), C.byref(ms)) == L.EINVAL
    assert b"window" in lib.sim_last_error(None)


def test_null_handles(lib):
    assert lib.sim_step(None, 1) == L.EINVAL
    assert lib.sim_sync(None) == L.EINVAL
    assert lib.sim_now(None) == -1
    lib.sim_destroy(None)
    h = C.c_void_p(123)
    assert lib.sim_create(None, None, None, C.byref(h)) == L.EINVAL
    assert lib.sim_query_sizes(None, None) == L.EINVAL


def build_abi_client(td):
    """Compile tests/abi_client.c with gcc against include/dpsnn.h and link libdpsnn.so."""
    exe = os.path.join(td, "abi_client")
    libdir = os.path.dirname(L.LIB_PATH)
    subprocess.check_call(["gcc", "-std=c11", "-Wall", "-Werror", "-I" + os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "abi_client.c"), "-o", exe,
                           "-L" + libdir, "-ldpsnn", "-Wl,-rpath," + libdir])
    return exe


def test_c_program_links_the_library_and_gets_its_errors(lib):
    """A plain C program built against the header alone links libdpsnn.so and receives the
    documented error codes for bad configurations and NULL arguments (no GPU needed)."""
    with tempfile.TemporaryDirectory() as td:
        exe = build_abi_client(td)
        out = subprocess.run([exe, "errors"], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "errors ok"
