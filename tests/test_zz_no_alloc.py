"""The allocation-free brute-force kNN entry point against the workspace one:
two calls in a row on the same device (the second smaller, so the fixed
scratch holds the first call's contents when it starts), identical ids and
FP64 distances, and a clear error beyond the scratch's size."""
import numpy as np
import pytest

from paper_2602_21600_amd import workloads as W

pytestmark = pytest.mark.gpu


def _pair(X, Q, k):
    import torch
    from paper_2602_21600_amd import aqr
    Xd = torch.from_numpy(X).cuda()
    Qd = torch.from_numpy(Q).cuda()
    ref_id, ref_d, ref_c = aqr.aqr_knn_bruteforce(Xd, Qd, k)
    out_id = torch.full((Q.shape[0], k), -7, dtype=torch.int32, device="cuda")
    out_d = torch.zeros((Q.shape[0], k), dtype=torch.float64, device="cuda")
    cert = torch.zeros(Q.shape[0], dtype=torch.uint8, device="cuda")
    aqr.aqr_knn_bruteforce_noalloc(Xd, Qd, k, out_id, out_d, cert)
    torch.cuda.synchronize()
    return (ref_id.cpu().numpy(), ref_d.cpu().numpy(), ref_c.cpu().numpy(),
            out_id.cpu().numpy(), out_d.cpu().numpy(), cert.cpu().numpy())


def test_noalloc_equals_workspace_entry_point(orc):
    print("no-alloc kNN: two calls, the second smaller", flush=True)
    X, Q = W.tiny(20_000, 64, seed=41, clusters=9, nq=700)
    for nq, k in ((700, 20), (90, 7)):
        r_id, r_d, r_c, o_id, o_d, o_c = _pair(X, Q[:nq], k)
        np.testing.assert_array_equal(o_id, r_id)
        np.testing.assert_array_equal(o_d.view(np.uint64), r_d.view(np.uint64))
        np.testing.assert_array_equal(o_c, r_c)
    # and against the oracle on the smaller call
    rid, rd = orc.knn_f32(X, Q[:90], 7)
    np.testing.assert_array_equal(o_id, rid)


def test_noalloc_rejects_beyond_its_scratch():
    import torch
    from paper_2602_21600_amd import aqr
    cap = int(aqr.lib().aqr_knn_noalloc_max_bytes())
    X = torch.zeros((40_000, 8), dtype=torch.float32, device="cuda")
    nq = 64
    while aqr.aqr_knn_workspace_size(40_000, nq, 128) <= cap:
        nq *= 2
    Q = torch.zeros((nq, 8), dtype=torch.float32, device="cuda")
    out_id = torch.zeros((nq, 128), dtype=torch.int32, device="cuda")
    out_d = torch.zeros((nq, 128), dtype=torch.float64, device="cuda")
    with pytest.raises(aqr.AqrError, match="scratch"):
        aqr.aqr_knn_bruteforce_noalloc(X, Q, 128, out_id, out_d)
