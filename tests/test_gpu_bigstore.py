"""A synapse store beyond 2^34 records (needs an MI355X; about 180 GB of device memory).

The tile kernel addresses 16-byte pieces with 32-bit indices relative to the first piece of
each tile's source rows, and the spike history keeps 64-bit part starts, so the store may
outgrow 2^32 pieces (2^34 records, 64 GB).  The plain 128x128 grid (20.3M neurons, about 27G
records with the padding) is generated and stepped in the bench's launch; sampled synapse
rows, sampled pending inputs and one whole step of every neuron equal the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_1511_09325_amd import Simulation
from paper_1511_09325_amd import sim as S
from paper_1511_09325_amd import workloads as W

from test_gpu_fullsize import _check_rows, _sample_rows, _spot_step

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


@pytest.fixture(scope="module")
def big():
    import torch
    torch.cuda.empty_cache()
    p = W.grid(128, 128, 0)
    sizes = S.query_sizes(p)
    assert sizes["n_records"] > 2 ** 34
    free, _ = torch.cuda.mem_get_info()
    need = sum(int(sizes[k]) for k in ("synapse_bytes", "index_bytes", "state_bytes", "history_bytes"))
    if need > 0.9 * free:
        pytest.skip("needs %.0f GB of device memory, %.0f GB free" % (need / 1e9, free / 1e9))
    sim = Simulation(p, record_steps=61)
    yield p, sim
    sim.close()
    del sim
    torch.cuda.empty_cache()


def test_rows_beyond_2_34_records(big):
    p, sim = big
    n = sim.n_neurons
    rng = np.random.default_rng(128)
    # the last rows lie past 2^34 records
    rows = sorted(set(_sample_rows(p, n, rng, 16)) | {n - 2, n - 1 - p["npc"]})
    _check_rows(sim, p, rows)


@pytest.mark.parametrize("u", [30, 60])
def test_whole_steps_beyond_2_34_records(big, u):
    p, sim = big
    assert _spot_step(sim, p, u, np.random.default_rng(u), 300) > 0
