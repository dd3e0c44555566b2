"""Sorts enqueued under HIP graph capture (torch.cuda.graph) and replayed:
every replay must equal the eager result.  The library enqueues kernels
only (no memset nodes, no allocation when the caller passes a workspace), so
the whole sort is capturable."""
import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    import paper_1511_03404_amd as rs
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    rs.lib()
    return rs


def test_single_sort_graph_replay(rs):
    n = 300007
    keys = torch.from_numpy(datagen.keys("gaussian", n, 32, seed=3)).cuda()
    vals = torch.from_numpy(datagen.values(n, 32)).cuda()
    ctx = rs.context(0)
    ws = torch.empty(ctx.workspace_bytes(32, True, n), dtype=torch.uint8, device="cuda")
    ko, vo = torch.empty_like(keys), torch.empty_like(vals)
    rs.sort_pairs(keys, vals, ko, vo, workspace=ws)
    torch.cuda.synchronize()
    want_k, want_v = ko.clone(), vo.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rs.sort_pairs(keys, vals, ko, vo, workspace=ws)
    for i in range(3):
        ko.zero_()
        vo.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(ko, want_k) and torch.equal(vo, want_v), f"replay {i}"
        # unrelated eager work between replays, through the same library
        rs.sort_keys(keys[: n // 3])
        torch.cuda.synchronize()


def test_segmented_graph_replay(rs):
    k, v, off = datagen.segmented(num_segments=400, lo_log2=4, hi_log2=17, bits=32, seed=9)
    kd, vd = torch.from_numpy(k).cuda(), torch.from_numpy(v).cuda()
    offd = torch.from_numpy(off.view(np.int64)).cuda()
    ctx = rs.context(0)
    ws = torch.empty(ctx.segmented_workspace_bytes(32, True, k.size, 400), dtype=torch.uint8,
                     device="cuda")
    ko, vo = torch.empty_like(kd), torch.empty_like(vd)
    rs.segmented_sort(kd, vd, offd, ko, vo, workspace=ws)
    torch.cuda.synchronize()
    want_k, want_v = ko.clone(), vo.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rs.segmented_sort(kd, vd, offd, ko, vo, workspace=ws)
    for i in range(3):
        ko.fill_(7)
        vo.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(ko, want_k) and torch.equal(vo, want_v), f"replay {i}"
