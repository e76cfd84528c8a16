"""The allocation-free forward pass (gsls_ws_forward_static) against the
handle-workspace one (gsls_ws_forward): the same kernels on the same inputs,
so the outputs agree bit for bit, on two calls in a row (the second with
fewer rows, in the workspace the first one left), and rows beyond the fixed
workspace are refused."""
import numpy as np
import pytest

from paper_2604_07644_amd import workloads as W

pytestmark = pytest.mark.gpu

from paper_2604_07644_amd import gsls  # noqa: E402  (fails loudly without libgsls.so)
import torch  # noqa: E402


def test_forward_static_matches_forward():
    ws = gsls.WarmStart(W.ws_init(21).astype(np.float32), W.ws_sketch().astype(np.float32))
    rng = np.random.default_rng(22)
    for rows in (2048, 777):
        X = torch.tensor(rng.standard_normal((rows, 160)) * 0.8, dtype=torch.float32, device="cuda").to(torch.bfloat16)
        ref = ws.forward(X).cpu().numpy()
        got = ws.forward_static(X).cpu().numpy()
        assert got.shape == ref.shape == (rows, 192)
        np.testing.assert_array_equal(got, ref)
    X = torch.zeros((2049, 160), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(gsls.GslsError) as e:
        ws.forward_static(X)
    assert e.value.code == gsls.ERR_DIM
    ws.close()
