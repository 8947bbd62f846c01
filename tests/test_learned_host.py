"""Host logic of the learned form's training driver (no GPU)."""
import numpy as np
import torch

from paper_2212_05645_amd.learned import balanced_epoch


def test_balanced_epoch_draws_every_decision_equally():
    g = torch.Generator().manual_seed(3)
    flags = torch.tensor([0] * 500 + [1] * 13 + [-1] * 70, dtype=torch.int8)
    pool = torch.arange(len(flags), dtype=torch.int32)[::2].contiguous()      # a subset of the rows
    order = balanced_epoch(flags, pool, g, torch)
    lab = flags[order.long()]
    counts = [int((lab == c).sum()) for c in (0, 1, -1)]
    assert counts[0] == counts[1] == counts[2] == int((flags[pool.long()] == 0).sum())
    assert set(order.tolist()) <= set(pool.tolist())
    # the largest class appears once each, in a shuffled order
    keep = order[lab == 0]
    assert sorted(keep.tolist()) == sorted(pool[flags[pool.long()] == 0].tolist())
    again = balanced_epoch(flags, pool, torch.Generator().manual_seed(3), torch)
    assert torch.equal(order, again)


def test_balanced_epoch_skips_absent_classes():
    g = torch.Generator().manual_seed(0)
    flags = torch.tensor([0] * 10 + [1] * 3, dtype=torch.int8)
    order = balanced_epoch(flags, torch.arange(13, dtype=torch.int32), g, torch)
    lab = flags[order.long()]
    assert len(order) == 20 and int((lab == 1).sum()) == 10 and int((lab == -1).sum()) == 0
