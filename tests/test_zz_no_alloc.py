"""The no-allocation query entry point (fclsh_query_batch_noalloc), called
through the C ABI, against fclsh_query_batch_async on the same inputs: two
calls in a row, the second with a smaller batch, must give the same offsets,
ids and status as the allocating path, and a batch too large for the fixed
scratch is refused before anything runs."""
import ctypes
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1602_02620_amd as fc  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def _run(fn, idx, q, r, radii, stream, cap):
    nq = q.shape[0]
    offsets = torch.full((nq + 1,), -1, dtype=torch.int64, device="cuda")
    ids = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    result = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    rp = _vp(radii) if radii is not None else ctypes.c_void_p()
    st = fn(idx._h, _vp(q), nq, r, rp, ctypes.c_void_p(stream.cuda_stream), _vp(offsets), _vp(ids), cap,
            _vp(result))
    assert st == fc.FCLSH_OK, fc.lib().fclsh_last_error().decode()
    stream.synchronize()
    total, status = (int(x) for x in result.cpu())
    return offsets.cpu().numpy(), ids[:max(total, 0)].cpu().numpy(), total, status


def test_noalloc_matches_async():
    w = synth.mid(0.02)  # 20,000 uniform 256-bit points, r = 8, L = 511
    _say(f"[noalloc] n={w.n} d={w.d} r={w.r} nq={w.nq}")
    idx = fc.Index(fc.to_device_words(w.points), w.d, w.r, seed=11)
    lib = fc.lib()
    stream = torch.cuda.Stream()
    q_all = fc.to_device_words(np.concatenate([w.queries] * 4))
    radii_all = torch.from_numpy(np.random.default_rng(3).integers(0, w.r + 1, q_all.shape[0]).astype(np.int32)).cuda()
    idx.reserve(q_all.shape[0], pair_capacity=1 << 16, spill_capacity=1 << 14, stream=stream)
    for nq, radii in ((q_all.shape[0], radii_all), (7, None)):  # the second call smaller
        q = q_all[:nq].contiguous()
        rad = radii[:nq].contiguous() if radii is not None else None
        want = _run(lib.fclsh_query_batch_async, idx, q, w.r, rad, stream, 1 << 16)
        got = _run(lib.fclsh_query_batch_noalloc, idx, q, w.r, rad, stream, 1 << 16)
        _say(f"[noalloc] nq={nq}: total {got[2]} status {got[3]}")
        assert want[3] == 0 and got[3] == 0
        assert got[2] == want[2]
        assert np.array_equal(got[0], want[0])
        assert np.array_equal(got[1], want[1])
    # a batch whose keys alone exceed the fixed scratch is refused up front
    L = idx.info["L"]
    too_many = (64 << 20) // (4 * L) + 1
    big = torch.zeros((too_many, fc.words(w.d)), dtype=torch.int64, device="cuda")
    offs = torch.zeros(too_many + 1, dtype=torch.int64, device="cuda")
    res = torch.zeros(2, dtype=torch.int64, device="cuda")
    st = lib.fclsh_query_batch_noalloc(idx._h, _vp(big), too_many, w.r, ctypes.c_void_p(),
                                       ctypes.c_void_p(stream.cuda_stream), _vp(offs), ctypes.c_void_p(), 0, _vp(res))
    assert st == fc.FCLSH_ENOMEM
    idx.close()
