"""Serving loop on the GPU: batches that overlap on several streams, admitted
by slots and output memory, give the same rows as each batch run alone and
as the oracle (mixed radius / K-NN rows, bit for bit)."""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_cs_0608108_amd import sphidx
    sphidx.load()
    return sphidx


def _rows_equal(a, b, what):
    rp_a, ids_a = a
    rp_b, ids_b = b
    assert np.array_equal(np.asarray(rp_a), np.asarray(rp_b)), what + ": row_ptr"
    assert np.array_equal(np.asarray(ids_a)[: int(rp_a[-1])], np.asarray(ids_b)[: int(rp_b[-1])]), what + ": ids"


@pytest.mark.parametrize("slots,pool_mb", [(3, 64), (4, 1)])
def test_batches_in_the_mix_equal_alone_and_oracle(sx, orc, slots, pool_mb):
    from paper_cs_0608108_amd import serving, synth
    spec = synth.LatticeSpec((6, 6, 6), 16, 7)
    n = 150000
    pts = synth.uniform_points(spec, n, 21)
    lat = sx.Lattice(spec.log2_cells, spec.frac_bits, spec.cyclic_mask, n)
    dev = [sx.to_dev_u32(a) for a in pts]
    lat.build(*dev)
    tab = sx.Tables(lat, 2, 4 * spec.edge)
    sizes = synth.serving_batch_sizes(21, 14, 2048)
    batches = []
    for i, s in enumerate(sizes):
        q, r, k = synth.serving_batch(spec, 21, i, int(s), rmin_k=64, rmax_k=256, knn_cap_cells=4)
        batches.append(serving.Batch(i, 0.0, q, r, k))
    say(f"serving slots={slots} pool={pool_mb} MB sizes={list(map(int, sizes))}")
    ex = serving.GpuExecutor(lat, tab, slots, int(max(sizes)), pool_mb << 20)
    serving.run_admission_model(batches, ex, slots, pool_mb << 20, keep=True)
    L = orc.Lattice(spec.log2_cells, spec.frac_bits, spec.cyclic_mask)
    g = orc.Grid(L, pts)
    alone = [serving.Batch(b.index, 0.0, b.centres, b.radius, b.k) for b in batches]
    serving.one_launch_per_batch(alone, lat, tab, keep=True)
    for b, a in zip(batches, alone):
        ref = g.mixed(b.k, b.radius, queries=b.centres)
        if b.rejected:
            assert 4 * int(ref.row_ptr[-1]) > (pool_mb << 20), b.index
            continue
        _rows_equal(b.result, (ref.row_ptr, ref.ids), f"batch {b.index} in the mix vs oracle")
        _rows_equal(a.result[:2], (ref.row_ptr, ref.ids), f"batch {b.index} alone vs oracle")
    g.close()
    assert sum(not b.rejected for b in batches) >= len(batches) - 2
