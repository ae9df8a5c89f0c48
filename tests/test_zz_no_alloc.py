"""Allocation-free scoring entry point (hgp_mlp_score_device_noalloc) against
hgp_mlp_score_device, through the C-ABI: identical int64 scores on two calls
in a row, the second with fewer rows (the scratch keeps the first call's
contents), plus its size limit.  The integer network is exact on MFMA, so
the comparison is exact; the oracle's scores pin both."""
import sys

import numpy as np
import pytest

import oracle
from paper_2604_14411_amd.synth import feature_codes, random_int_mlp

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32)).to("cuda:0")


def test_noalloc_scoring_matches_allocating_entry_point():
    import torch

    from paper_2604_14411_amd import hgp

    assert torch.cuda.is_available()
    ctx = hgp.Context(0)
    try:
        for call, (seed, n) in enumerate([(1, 70001), (2, 1237)]):
            q = random_int_mlp(500 + seed)
            x = feature_codes(600 + seed, n)
            xd = _dev(x)
            say(f"[noalloc] call {call} rows={n}")
            ref = hgp.mlp_score_device(ctx, q, xd).cpu().numpy()
            out = torch.full((n,), -7, dtype=torch.int64, device="cuda:0")
            got = hgp.mlp_score_device_noalloc(ctx, q, xd, out=out).cpu().numpy()
            assert np.array_equal(got, ref), f"call {call}"
            assert np.array_equal(got, oracle.mlp_score(q, x)), f"call {call}"
        say("[noalloc] limits")
        import ctypes

        # more rows than the scratch holds: rejected on the host before any
        # launch (the buffers passed are real, small device tensors)
        xs = _dev(np.zeros((4, 16)))
        os_ = torch.empty(4, dtype=torch.int64, device="cuda:0")
        m = hgp.mlp_struct(random_int_mlp(1))
        rc = hgp.load().hgp_mlp_score_device_noalloc(ctx.handle, ctypes.byref(m), xs.data_ptr(),
                                                     hgp.NOALLOC_MAX_ROWS + 1, os_.data_ptr(), hgp._stream())
        assert rc == hgp.EUNSUPPORTED
        assert b"HGP_NOALLOC_MAX_ROWS" in hgp.load().hgp_last_error()
        assert hgp.mlp_score_device_noalloc(ctx, random_int_mlp(1), _dev(np.zeros((0, 16)))).numel() == 0
    finally:
        ctx.close()
