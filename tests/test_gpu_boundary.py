"""The C ABI boundary on the GPU: a plain C program and caller-owned (torch) device memory.

* tests/abi_client.c, built with gcc against include/dpsnn.h alone, runs the whole 2x2
  workload (1 s) through sim_query_sizes / sim_create / sim_step / sim_read_spikes /
  sim_get_stats; its raster and counters equal the oracle's.
* The same workload built on torch-owned buffers for all four regions that sim_query_sizes
  sizes (synapses, index, state, history) is bit-exact against the oracle, and the state
  region read through torch views equals sim_read_state.
* sim_backward (built-in loss of the column rates against targets) equals sim_backward_rates
  fed with that loss's gradient.
"""
import ctypes as C
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from paper_1511_09325_amd import _lib as L
from paper_1511_09325_amd import Simulation
from paper_1511_09325_amd import sim as S
from paper_1511_09325_amd import workloads as W

from test_abi import build_abi_client

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


_FIELDS = ("npc", "n_exc", "d_min", "d_max", "t_ref", "ext_syn", "p_own", "p_remote", "decay_um",
           "spacing_um", "we_mu", "we_sigma", "wi_mu", "wi_sigma", "tau_m", "theta", "v_reset",
           "tau_ca", "ca_inc", "g_ahp", "dt", "j_ext", "rows", "cols", "seed", "ext_rate_hz")


def _oracle_run(p, T):
    ref = oracle.Sim(p)
    ref.step(T)
    return ref


def test_c_program_runs_the_2x2_workload():
    p, T = W.PLAIN_2X2["params"], W.PLAIN_2X2["steps"]
    with tempfile.TemporaryDirectory() as td:
        exe = build_abi_client(td)
        args = [exe, "run", str(T)] + ["%s=%r" % (k, p[k]) for k in _FIELDS]
        out = subprocess.run(args, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    lines = out.stdout.strip().splitlines()
    assert len(lines) == T + 1
    ref = _oracle_run(p, T)
    for u, line in enumerate(lines[:T]):
        f = line.split()
        assert f[0] == "step" and int(f[1]) == u and int(f[2]) == len(f) - 3
        assert np.array_equal(np.array(f[3:], np.int64), ref.spikes(u)), u
    c = ref.counts()
    assert lines[T].split()[1:] == [str(c["spikes"]), str(c["e_rec"]), str(c["e_ext"])]


ALL = ("synapses", "index", "state", "history")


def test_torch_owned_buffers_2x2_workload_bit_exact():
    import torch
    p, T = W.PLAIN_2X2["params"], W.PLAIN_2X2["steps"]
    sizes = S.query_sizes(p, record_steps=T, raster_capacity=T * 4960)
    lib_sim = Simulation(p, record_steps=T, raster_capacity=T * 4960)
    sim = Simulation(p, record_steps=T, raster_capacity=T * 4960, torch_buffers=ALL)
    assert sim.sizes == sizes
    want = sum(int(sizes[k]) for _, k in L.REGIONS)
    assert sim.caller_bytes == want
    assert all(int(sim.buffers[n].numel()) == int(sizes[k]) for n, k in L.REGIONS)
    # the library holds what it held before minus the four regions (each region rounds its
    # arrays up to 256-byte offsets)
    extra = sim.device_bytes + want - lib_sim.device_bytes
    assert 0 <= extra <= 256 * 16, extra
    assert lib_sim.digest() == sim.digest()
    del lib_sim
    sim.step(T)
    sim.sync()
    ref = _oracle_run(p, T)
    got = sim.read_spikes(0, 0, T)
    for u in range(T):
        assert np.array_equal(got[u], ref.spikes(u)), u
    a, b = sim.state(0), ref.state()
    for k in ("v", "ca", "ref", "pend"):
        assert np.array_equal(a[k], b[k]), k
    v, ca, rf = sim.state_tensors()
    assert np.array_equal(v.cpu().numpy(), a["v"])
    assert np.array_equal(ca.cpu().numpy(), a["ca"])
    assert np.array_equal(rf.cpu().numpy(), a["ref"])
    st, rc = sim.stats(0), ref.counts()
    assert (st["spikes"], st["e_rec"], st["e_ext"]) == (rc["spikes"], rc["e_rec"], rc["e_ext"])
    sim.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("regions", [("state",), ("synapses", "history")])
def test_some_regions_torch_owned(regions):
    p = W.tiny(3, 2, npc=44, seed=12)
    T = 80
    a = Simulation(p, record_steps=T, torch_buffers=regions)
    b = Simulation(p, record_steps=T)
    a.step(T)
    b.step(T)
    assert a.digest() == b.digest()
    assert all(np.array_equal(x, y) for x, y in zip(a.read_spikes(), b.read_spikes()))


def test_caller_buffers_too_small_or_misaligned_are_refused():
    import torch
    p = W.tiny(2, 2, npc=40, seed=2)
    cfg, nets = S.make_config(p)
    sizes = S.query_sizes(p)
    lib = L.lib()
    t = torch.empty(int(sizes["state_bytes"]) + 512, dtype=torch.uint8, device="cuda")
    for ptr, nbytes, msg in ((t.data_ptr(), int(sizes["state_bytes"]) - 256, b"needs"),
                             (t.data_ptr() + 16, int(sizes["state_bytes"]), b"aligned")):
        bufs = L.SimBuffers()
        bufs.state, bufs.state_bytes = C.c_void_p(ptr), nbytes
        h = C.c_void_p()
        assert lib.sim_create(C.byref(cfg), C.byref(bufs), None, C.byref(h)) == L.EINVAL
        assert h.value is None
        assert msg in lib.sim_last_error(None)


def test_backward_with_builtin_loss_equals_backward_of_its_gradient():
    import torch
    p = W.tiny(2, 3, npc=40, seed=3, ext_rate_hz=3.4)
    T = 90
    sim = Simulation(p, train_mode=True, ckpt_every=30, surrogate_beta=5.0)
    sim.step(T)
    rates = sim.column_rates().cpu().numpy()
    tg = np.random.default_rng(4).uniform(2.0, 8.0, size=sim.n_cols).astype(np.float32)
    loss, gw, gt, gg = sim.backward_loss(tg)
    d = rates.astype(np.float64) - tg.astype(np.float64)
    want_loss = float(np.mean(d * d))
    assert abs(loss - want_loss) <= 1e-6 * want_loss
    gr = (2.0 * d / len(d)).astype(np.float32)
    gw2, gt2, gg2 = sim.backward(torch.tensor(gr, device="cuda"))
    assert torch.equal(gw, gw2) and (gt, gg) == (gt2, gg2)
    assert float(gw.abs().sum()) > 0
