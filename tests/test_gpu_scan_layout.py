"""Column layout of the scans (ohm_map_set_scan_layout): the grouped walk
takes 8-beam by 32-column patches of a column-major range image as its
tiles.  Only the walk order changes, so every result must be the given
order's: bit-identical occupancy, counts and statistics against the oracle
in count mode with unit weights; the same bits as the given order with
exactly summable weights and with the mean and decay-rate layers (integer
sums).  Scans hold whole 32-column chunks, a partial last chunk (walked in
the given order) or less than one chunk, and the declared layout matches
the data (64 rays per column) or not (8 and 136: the order is a bijection
for any multiple of 8)."""
import numpy as np
import pytest

import oracle
import paper_2206_06079_amd as ohm
from gpu_helpers import device, to_dev
from workloads import scenes
from workloads.scenes import RayBatch

pytestmark = pytest.mark.gpu

GROUPED = ohm.LAYER_OCC | ohm.LAYER_SCAN_GROUPS
BOX_MIN = (690, 978, 183)
BOX_DIM = (720, 44, 34)
# rays kept of each of 11 spinning-lidar scans (131,072 = 64 chunks of
# 32 columns x 64 beams): whole, ragged by a few rays or columns, shorter
# than a chunk, one ray, empty
SIZES = (131072, 131072 - 700, 2047, 131072, 4096 + 5, 1, 0, 65536, 131072 - 64, 2048, 131072)


def ragged_batch():
    mp, full = scenes.config1(n_scans=len(SIZES), first_scan=40)
    parts = [full.samples[k * 131072:k * 131072 + n] for k, n in enumerate(SIZES)]
    offsets = np.concatenate([[0], np.cumsum(SIZES)]).astype(np.uint32)
    return mp, RayBatch(full.origins, np.concatenate(parts).astype(np.float32), offsets)


def run(mp, batch, layers, col_rays, capacity=1024):
    m = ohm.OhmMap(mp, capacity, layers=layers, device=device())
    m.set_scan_layout(col_rays)
    o, s, off, w = to_dev(batch)
    m.integrate(o, s, off, w)
    out = {"occ": m.read_dense(ohm.READ_OCC, BOX_MIN, BOX_DIM).cpu().numpy(),
           "hits": m.read_dense(ohm.READ_HITS, BOX_MIN, BOX_DIM).cpu().numpy(),
           "miss": m.read_dense(ohm.READ_MISSES, BOX_MIN, BOX_DIM).cpu().numpy(), "stats": m.stats()}
    if layers & ohm.LAYER_MEAN:
        out["packed"] = m.read_dense(ohm.READ_MEAN_PACKED, BOX_MIN, BOX_DIM).cpu().numpy().view(np.uint32)
        out["count"] = m.read_dense(ohm.READ_MEAN_COUNT, BOX_MIN, BOX_DIM).cpu().numpy().view(np.uint32)
    if layers & ohm.LAYER_DECAY:
        out["length"] = m.read_dense(ohm.READ_DECAY_LENGTH, BOX_MIN, BOX_DIM).cpu().numpy()
        out["dhits"] = m.read_dense(ohm.READ_DECAY_HITS, BOX_MIN, BOX_DIM).cpu().numpy().view(np.uint32)
    m.close()
    return out


@pytest.fixture(scope="module")
def ragged():
    mp, batch = ragged_batch()
    print(f"layout: scans of {SIZES} rays", flush=True)
    return mp, batch, oracle.integrate_count(mp, batch, BOX_MIN, BOX_DIM)


@pytest.mark.parametrize("col_rays", [64, 8, 136])
def test_layout_equals_oracle(ragged, col_rays):
    """Groups of 8 scans and a last group of 3, with empty and one-ray scans
    among them."""
    mp, batch, (o_occ, o_hit, o_miss, o_st) = ragged
    g = run(mp, batch, GROUPED, col_rays)
    assert np.count_nonzero(o_occ) > 100_000
    assert np.array_equal(g["occ"], o_occ)
    assert np.array_equal(g["hits"], o_hit) and np.array_equal(g["miss"], o_miss)
    st = g["stats"]
    assert st["voxel_updates"] == o_st["updates"]
    assert st["rays_in"] == o_st["rays"] and st["rays_truncated"] == o_st["truncated"]
    assert st["updates_dropped_pool"] == 0


def test_layout_weighted_and_layers_match_given_order(ragged):
    """Weights from {0.5, 0.75, 1} (exact Q32.32 sums) through the grouped
    walk, and the mean and decay-rate layers together: the same bits with
    and without the layout."""
    mp, batch, _ = ragged
    wb = RayBatch(batch.origins, batch.samples, batch.offsets,
                  np.random.default_rng(21).choice(np.float32([0.5, 0.75, 1.0]), batch.n_rays))
    for b, layers in ((wb, GROUPED), (batch, GROUPED | ohm.LAYER_MEAN | ohm.LAYER_DECAY)):
        a = run(mp, b, layers, 0)
        c = run(mp, b, layers, 64)
        for key in a:
            if key == "stats":
                assert a[key]["voxel_updates"] == c[key]["voxel_updates"]
                assert a[key]["rays_hit"] == c[key]["rays_hit"]
            else:
                assert np.array_equal(a[key], c[key]), key


def test_layout_arguments_checked():
    mp, _ = scenes.config1(n_scans=1)
    m = ohm.OhmMap(mp, 8, layers=GROUPED, device=device())
    for bad in (7, 12, 65544):
        with pytest.raises(RuntimeError):
            m.set_scan_layout(bad)
    for good in (0, 8, 64, 65536):
        m.set_scan_layout(good)
    m.close()
