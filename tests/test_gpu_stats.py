"""Walk statistics (FP64 rechecks, child levels descended): consistent
across the walks that visit the same leaves, and zero where no descent can
occur."""
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

import paper_1311_0705_amd as hg  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def disk():
    w = W.workload(2)
    w.criteria.delta_max = 1e-5
    g = hg.build(w.density, w.criteria, w.tree_type, device=DEV)
    o, k = W.rays(w.ray_kind, 200_000, w.ray_seed)
    yield g, torch.from_numpy(o).to(DEV), torch.from_numpy(k).to(DEV)
    g.free()


def test_descents_agree_across_walks(disk):
    g, o, k = disk
    runs = []
    for prec in (hg.FP64, hg.FP32_RECHECK):
        for mode, passes in ((hg.TAU_ONLY, 0), (hg.RECORDS, 1), (hg.RECORDS, 2)):
            for persistent in (0, 3):
                r = g.trace(o, k, precision=prec, mode=mode, passes=passes, persistent=persistent,
                            count_rechecks=True)
                runs.append((prec, mode, passes, persistent, r["descents"], r["rechecks"]))
    d = {x[4] for x in runs}
    assert len(d) == 1 and d.pop() > 0, runs
    # FP64 never rechecks; the FP32 walk does the same number of times whatever the mode
    assert all(x[5] == 0 for x in runs if x[0] == hg.FP64)
    assert len({x[5] for x in runs if x[0] == hg.FP32_RECHECK}) == 1
    # the batched walk over one grid counts the same
    rb = hg.trace_batched([g], [o], [k], precision=hg.FP32_RECHECK, mode=hg.TAU_ONLY, count_rechecks=True)
    assert rb[0]["descents"] == runs[0][4]


def test_no_descent_on_a_regular_octree():
    # uniform density, mass criterion: every leaf at level 5, so ropes end in
    # leaves and a locate-table cell at depth >= 5 is a leaf or inside one
    d = W.Density(box=(-1, -1, -1, 1, 1, 1, 1.0))
    cr = W.Criteria(total_mass=W.total_mass(d), delta_max=1e-4, max_level=5, seed=3)
    g = hg.build(d, cr, W.OCTREE, device=DEV)
    assert g.n_leaves == 32768
    o, k = W.rays("uniform", 20000, 5)
    # 32768 leaves give a locate table of depth 5: its cells are the leaves
    for persistent in (0, 3):
        r = g.trace(o, k, precision=hg.FP64, mode=hg.TAU_ONLY, count_rechecks=True, persistent=persistent)
        assert r["descents"] == 0
        assert int(r["count"].sum().item()) > 20000
    g.free()
