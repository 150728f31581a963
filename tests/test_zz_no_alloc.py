"""The packing entry point that allocates nothing (hc_pack_run_static, for
callers that cannot allocate device memory) against the workspace entry
point hc_pack_run: the same iterations must give the same centres and the
same overlap record bit for bit, on two calls in a row, the second with
fewer ellipsoids (the static scratch keeps the first call's contents)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _rots(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1)], 1)


def _inputs(seed, n, box, semi):
    rng = np.random.default_rng(seed)
    c = (rng.uniform(0, 1, (n, 3)) * np.asarray(box)).astype(np.float32)
    R = _rots(rng, n).astype(np.float32).reshape(n, 9)
    s = np.tile(np.asarray(semi, dtype=np.float32), (n, 1)) * rng.uniform(0.8, 1.0, (n, 1)).astype(np.float32)
    return c, R, s


def test_static_packing_matches_workspace_packing():
    import torch

    from paper_2305_02752_amd import Packer
    semi = (8.5, 8.5, 3.8)
    for seed, n, side in ((71, 400, 150.0), (72, 90, 100.0)):   # the second call is smaller
        box = (side, side, side)
        pk = Packer(box, (True, True, True), max_semi=8.5, eta=0.03, max_move=1.0, quad=8)
        c, R, s = _inputs(seed, n, box, semi)
        dev = torch.device("cuda:0")
        ta = torch.tensor(c, device=dev)
        tb = torch.tensor(c, device=dev)
        tr = torch.tensor(R, device=dev)
        ts = torch.tensor(s, device=dev)
        ra = pk.run_device(ta, tr, ts, 6)
        rb = pk.run_device_static(tb, tr, ts, 6)
        torch.cuda.synchronize()
        a, b = ta.cpu().numpy(), tb.cpu().numpy()
        print(f"n={n}: overlap {ra} vs {rb}", flush=True)
        assert np.array_equal(a, b)
        assert ra == rb
        assert not np.array_equal(a, c)     # the iterations moved the ellipsoids
