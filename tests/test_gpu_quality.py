"""The zonal-coding quality sweep (Section 3's experiment on synthetic images):
the GPU's per-image squared error equals the oracle's exactly for every r,
and the bench's DCT reference is the orthonormal DCT-II."""
import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def test_sweep_sse_matches_oracle():
    import torch
    import paper_1702_00817_amd as tdct
    side, rs = 512, [2, 6, 10, 25, 35, 45]
    one = np.ones(64, np.uint16)
    for i in range(3):
        img = synth.plane(side, side, 100 + i)
        src = torch.from_numpy(img).cuda()
        dst = torch.empty_like(src)
        sse = torch.zeros(len(rs), dtype=torch.int64, device="cuda")
        for k, r in enumerate(rs):
            tdct.tdct_roundtrip(src, side, side, side, one, r, None, dst, side)
            tdct.tdct_sse(src, side, dst, side, side, side, sse[k].data_ptr())
        torch.cuda.synchronize()
        for k, r in enumerate(rs):
            _, rec = O.roundtrip(img, one, r)
            assert int(sse[k].item()) == O.sse(img, rec), (i, r)
