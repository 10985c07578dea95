"""cm_geometry_destroy through the C ABI (needs an MI355X): destroyed ids stay
reserved and are refused, the other geometries keep their ids and their
results, the vertex pool is repacked."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import cm_oracle as O
from tests.parity import compare_outputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_destroy_geometry():
    from paper_2602_20304_amd.cm import Context
    from paper_2602_20304_amd._lib import CMError
    ctx = Context(0)
    b = W.mixed_scenes(24, seed=31)
    ids = ctx.create_geometry(b.geoms)
    pool0 = ctx.vertex_pool_size
    # destroy the geometries of scenes 12..23 (bodies 96..191)
    dead = np.unique(ids[b.body_geom[96:]])
    live = np.setdiff1d(ids, dead)
    info_before = {int(g): ctx.geometry_info(int(g)) for g in live}
    _say(f"[gpu] destroy {len(dead)} of {len(ids)} geometries")
    ctx.destroy_geometry(dead)
    assert ctx.geometry_count == len(ids)
    assert ctx.vertex_pool_size == sum(info_before[int(g)]["n_vertices"] for g in live) < pool0
    for g in dead[:3]:
        with pytest.raises(CMError) as e:
            ctx.geometry_info(int(g))
        assert e.value.status == -6
    with pytest.raises(CMError) as e:
        ctx.destroy_geometry(dead[:1])
    assert e.value.status == -6
    for g in live:
        i = ctx.geometry_info(int(g))
        for k in ("type", "n_vertices", "n_edges", "n_faces"):
            assert i[k] == info_before[int(g)][k]
    # the surviving scenes still match the oracle
    keep = W.subset_scenes(b, np.arange(12))
    db = ctx.upload_batch(keep, ids)
    m = ctx.collide(db, keep.tau, keep.K)
    ctx.check_errors()
    got = m.to_numpy()
    pairs, off = O.broadphase(keep)
    assert np.array_equal(got["pairs"], pairs) and np.array_equal(got["offsets"], off)
    _, _, ref = O.collide_batch(keep, pair_list=pairs)
    ok, rep = compare_outputs(got, ref)
    assert ok, rep
    # a batch that references a destroyed geometry is flagged
    gone = W.subset_scenes(b, np.arange(12, 14))
    db2 = ctx.upload_batch(gone, ids)
    ctx.collide(db2, gone.tau, gone.K)
    with pytest.raises(CMError) as e:
        ctx.check_errors()
    assert e.value.status == -6
    ctx.close()
