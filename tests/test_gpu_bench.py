"""The benchmark's choice between two launch-shape pairs in whole encode +
decode steps: both pairs' plans run on the GPU over the same batch, the
call returns one of them with a positive median step time each, and the
batch's outputs are then the oracle's (the pairs did the same work)."""
import numpy as np
import pytest

import bench
import oracle as O
import synth

pytestmark = pytest.mark.gpu


def test_step_choice_runs_both_pairs_and_outputs_stay_exact():
    import torch

    import paper_1702_00817_amd as tdct
    W = bench.make_large_batch(tdct, torch, 4, 512)
    ref = tuple(bench.parse_tune(x) for x in bench.REFERENCE_TUNE.split(":"))
    other = (bench.parse_tune("1,4096,1,0,0"), bench.parse_tune("8,1,1,1,1"))
    stream = torch.cuda.current_stream()
    k, med = bench.step_choice(tdct, torch, W, [ref, other], stream, rounds=2, steps=3)
    torch.cuda.synchronize()
    assert k in (0, 1) and len(med) == 2 and all(m > 0 for m in med)
    for i in range(4):
        w, h = W["sizes"][i]
        img = synth.batch_view(W["buf"], W["off"], W["strides"], W["sizes"], i)
        q = O.quantise(img, W["qs"][i], 64)
        assert np.array_equal(W["coef"][i].cpu().numpy(), q)
        assert np.array_equal(W["dst"][i].cpu().numpy(), O.inverse(q, W["qs"][i], w, h))
