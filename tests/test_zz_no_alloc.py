"""bpfa_set_state_noalloc, the state import that allocates nothing, against
bpfa_set_state through the C ABI.

Two handles share a frame and seed; one imports a state with bpfa_set_state,
the other with bpfa_set_state_noalloc (its temporary device memory in the
library's fixed buffer).  The imported states, read back, must be equal bit
for bit (the import is byte and index work), and so must one iteration run
from them.  Two imports in a row, the second smaller, show that the buffer's
leftover contents do not leak into the next call; an import that fails the
W / Z check followed by a valid one shows that the flag is cleared; a device
view passes through the C ABI with torch tensors; a host view larger than
the buffer is refused with ENOMEM and leaves the state unchanged.
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2311_15061_amd import bpfa  # noqa: E402

SCRATCH_BYTES = 32 << 20


def _frame(shape, rho, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    img = rng.random(shape).astype(np.float32)
    mask = (rng.random(shape) < rho).astype(np.uint8)
    return img, mask


def _state(N, K, P, density, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    D = (rng.standard_normal((K, P)) / np.sqrt(P)).astype(np.float32)
    Z = rng.random((N, K)) < density
    W = np.where(Z, rng.standard_normal((N, K)), 0.0).astype(np.float32)
    ell = rng.standard_normal(K) - 3.0
    return dict(D=D, W=W, Z=Z, logit_pi=ell, gamma_s=1.7, gamma_eps=55.0, t=4)


def _same(a, b):
    ga, gb = a.get_state(), b.get_state()
    for k in ("D", "W", "Z", "logit_pi"):
        assert np.array_equal(ga[k], gb[k]), k
    for k in ("gamma_s", "gamma_eps", "t"):
        assert ga[k] == gb[k], k
    return ga


def _pair_import(shape, patch, K, density, seed):
    img, mask = _frame(shape, 0.3, seed)
    ref = bpfa.Problem(img, mask, patch, K=K, seed=seed)
    new = bpfa.Problem(img, mask, patch, K=K, seed=seed)
    st = _state(ref.N, K, ref.P, density, seed + 1)
    assert 5 * ref.N * K + 256 <= SCRATCH_BYTES
    print("case: shape=%s patch=%s K=%d N=%d staged bytes=%d" % (shape, patch, K, ref.N, 5 * ref.N * K),
          flush=True)
    ref.set_state(**st)
    new.set_state(noalloc=True, **st)
    gs = _same(ref, new)
    assert np.array_equal(gs["W"], st["W"]) and np.array_equal(gs["Z"].astype(bool), st["Z"])
    ref.iterate(1)
    new.iterate(1)
    _same(ref, new)
    return ref, new


def test_noalloc_import_matches_set_state_twice_second_smaller():
    a = _pair_import((200, 200), (8, 8), 64, 0.1, 31)      # 11.9 MB staged
    b = _pair_import((48, 40), (6, 6), 24, 0.3, 32)        # the next call, 0.1 MB
    for p in (*a, *b):
        p.close()


def test_noalloc_flag_is_cleared_between_calls():
    img, mask = _frame((40, 40), 0.3, 7)
    ref = bpfa.Problem(img, mask, (8, 8), K=16, seed=7)
    new = bpfa.Problem(img, mask, (8, 8), K=16, seed=7)
    st = _state(ref.N, 16, ref.P, 0.2, 8)
    bad = dict(st)
    Zb = st["Z"].copy()
    r, c = np.argwhere(Zb)[0]
    Zb[r, c] = False          # W stays non-zero there
    bad["Z"] = Zb
    with pytest.raises(bpfa.BpfaError) as ei:
        new.set_state(noalloc=True, **bad)
    assert ei.value.status == bpfa.ESTATE
    ref.set_state(**st)
    new.set_state(noalloc=True, **st)   # the flag the failed call left set is cleared
    _same(ref, new)
    ref.close()
    new.close()


def test_noalloc_device_view_through_the_c_abi():
    import torch
    img, mask = _frame((36, 44), 0.3, 9)
    ref = bpfa.Problem(img, mask, (6, 6), K=20, seed=9)
    new = bpfa.Problem(img, mask, (6, 6), K=20, seed=9)
    st = _state(ref.N, 20, ref.P, 0.25, 10)
    ref.set_state(**st)
    dev = "cuda:0"
    D = torch.from_numpy(st["D"]).to(dev)
    W = torch.from_numpy(st["W"]).to(dev)
    Z = torch.from_numpy(st["Z"].astype(np.uint8)).to(dev)
    ell = torch.from_numpy(st["logit_pi"]).to(dev)
    torch.cuda.synchronize()
    v = bpfa.StateView(D=D.data_ptr(), W=W.data_ptr(), Z=Z.data_ptr(), logit_pi=ell.data_ptr(),
                       gamma_s=st["gamma_s"], gamma_eps=st["gamma_eps"], t=st["t"], mem=bpfa.DEVICE)
    assert bpfa.lib.bpfa_set_state_noalloc(new.handle, ctypes.byref(v)) == bpfa.OK
    _same(ref, new)
    ref.close()
    new.close()


def test_noalloc_refuses_host_views_beyond_its_buffer():
    img, mask = _frame((300, 300), 0.1, 12)
    p = bpfa.Problem(img, mask, (8, 8), K=128, seed=12)
    assert 5 * p.N * 128 > SCRATCH_BYTES
    before = p.get_state()
    st = _state(p.N, 128, p.P, 0.05, 13)
    with pytest.raises(bpfa.BpfaError) as ei:
        p.set_state(noalloc=True, **st)
    assert ei.value.status == bpfa.ENOMEM
    assert "fixed state-import buffer" in str(ei.value)
    after = p.get_state()
    for k in ("D", "W", "logit_pi"):
        assert np.array_equal(before[k], after[k]), k
    p.close()
