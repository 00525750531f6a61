"""The Python binding refuses short or mistyped buffers before any C call.

The C ABI takes raw device pointers and cannot see buffer sizes, so the
binding checks dtype and element counts against the call's layout (d
[B][ell][N], out [B][2][ell][N], the top-level key [ndig][2][key_ell+k][N],
the plan's workspace) and raises ValueError first. These tests run on the
host with CPU tensors and a parameter object whose handle is never used:
every case must raise before the binding reaches the library.
"""
import ctypes

import pytest
import torch

import paper_2603_16692_amd as ks


class _NoCall:
    """Stands in for the library: any call through it fails the test."""

    def __getattr__(self, name):
        raise AssertionError(f"the binding reached the library ({name}) before its checks")


def fake_params(dnum=2, log_n=5, ell=6, k=3, ws_bytes=4096):
    G = ks.KsParams.__new__(ks.KsParams)
    G._h = None
    G.n, G.log_n, G.ell, G.k = 1 << log_n, log_n, ell, k
    G.alpha, G.dnum = k, dnum
    G.ndig = -(-ell // k)
    G.key_ell = ell
    G.nl = ell + k
    G.workspace_bytes = lambda batch, plan=None: ws_bytes * max(batch, 1)
    G.eval_workspace_bytes = lambda batch, plan=None: 2 * ws_bytes * max(batch, 1)
    return G


@pytest.fixture
def no_lib(monkeypatch):
    monkeypatch.setattr(ks, "_lib", _NoCall())


def words(*shape, dtype=torch.int64):
    return torch.zeros(shape, dtype=dtype)


def test_keyswitch_rejects_short_and_mistyped_buffers(no_lib):
    G = fake_params()
    B, n, ell, nl = 2, G.n, G.ell, G.nl
    d, out = words(B, ell, n), words(B, 2, ell, n)
    evk = words(G.ndig, 2, nl, n)
    ws = words(2 * 4096 // 8)
    cases = [
        (words(B, ell, n - 1), evk, out, ws, "d"),
        (d, words(G.ndig, 2, nl - 1, n), out, ws, "evk"),
        (d, evk, words(B, 2, ell, n)[:, :1].contiguous(), ws, "out"),
        (d, evk, out, words(2 * 4096 // 8 - 1), "ws"),
        (words(B, ell, n, dtype=torch.int32), evk, out, ws, "d"),
        (d, evk.to(torch.float64), out, ws, "evk"),
    ]
    for dd, ee, oo, ww, what in cases:
        with pytest.raises(ValueError, match=what):
            G.keyswitch(dd, ee, oo, B, ww)
    # a batch larger than the buffers were made for
    with pytest.raises(ValueError, match="d"):
        G.keyswitch(d, evk, out, B + 1, words(8 * 4096))
    # the checks would pass: the next step is the library, which must not be reached here
    with pytest.raises(AssertionError, match="reached the library"):
        G.keyswitch(d, evk, out, B, ws)


def test_step_calls_check_their_layouts(no_lib):
    G = fake_params()
    B, n, ell, nl, nd = 3, G.n, G.ell, G.nl, G.ndig
    G._staged_ws_bytes = lambda batch: 1024 * batch
    ws = words(3 * 1024 // 8)
    with pytest.raises(ValueError, match="ext"):
        G.modup(words(B, ell, n), words(B, nd, nl, n - 1), B, ws)
    with pytest.raises(ValueError, match="ws"):
        G.modup(words(B, ell, n), words(B, nd, nl, n), B, words(10))
    with pytest.raises(ValueError, match="acc"):
        G.keymult(words(B, nd, nl, n), words(nd, 2, nl, n), words(B, 2, nl, n - 1), B)
    with pytest.raises(ValueError, match="evk"):
        G.keymult(words(B, nd, nl, n), words(nd, 2, nl - 1, n), words(B, 2, nl, n), B)
    with pytest.raises(ValueError, match="out"):
        G.moddown(words(B, 2, nl, n), words(B, 2, ell - 1, n), B, ws)
    with pytest.raises(ValueError, match="x"):
        G.ntt(words(B, 4, n - 1), 0, 4, B)
    with pytest.raises(ValueError, match="x"):
        G.intt(words(B, 4, n), 0, 4, B + 1)
    # BConv: digit 1 has alpha source limbs and nl - alpha targets; P has k sources, ell targets
    with pytest.raises(ValueError, match="src"):
        G.bconv(words(B, G.alpha - 1, n), 1, words(B, nl - G.alpha, n), B)
    with pytest.raises(ValueError, match="dst"):
        G.bconv(words(B, G.alpha, n), 1, words(B, nl - G.alpha - 1, n), B)
    with pytest.raises(ValueError, match="dst"):
        G.bconv(words(B, G.k, n), ks.KS_SET_P, words(B, ell - 1, n), B)


def test_hmul_hrot_and_graph_check_their_buffers(no_lib):
    G = fake_params()
    B, n, ell, nl = 2, G.n, G.ell, G.nl
    ct = words(B, 2, ell, n)
    evk = words(G.ndig, 2, nl, n)
    out = words(B, 2, ell, n)
    ews = words(2 * 2 * 4096 // 8)
    with pytest.raises(ValueError, match="b"):
        G.hmul(ct, words(B, 2, ell, n - 1), evk, out, B, ews)
    with pytest.raises(ValueError, match="d"):
        G.hmul(words(B, ell, n), ct, evk, out, B, ews)  # one component where two are read
    with pytest.raises(ValueError, match="ws"):
        G.hrot(ct, 5, evk, out, B, words(4096 // 8))  # a KeySwitch-sized workspace, not the eval one
    with pytest.raises(ValueError, match="out"):
        ks.Graph(G, words(B, ell, n), evk, words(B, ell, n), B, words(8 * 4096))


def test_level_handle_takes_the_top_level_key():
    # at a level the key keeps the top level's rows: [ndig_top][2][key_ell + k][N]
    G = fake_params(dnum=4, log_n=4, ell=5, k=2)
    G.key_ell = 8
    nd_top = -(-G.key_ell // G.alpha)
    assert G.shapes(1)["evk"] == (nd_top, 2, G.key_ell + G.k, G.n)
    assert G._key_words() == nd_top * 2 * (G.key_ell + G.k) * G.n


def test_abi_rejects_bad_parameters_without_a_device():
    # argument checks of ks_params_create come before any HIP call
    h = ctypes.c_void_p()
    for args in ((2, 18, 4), (1, 2, 4), (5, 12, 4), (0, 12, 4), (2, 10, 200)):
        assert ks.raw_call("ks_params_create", *args, ctypes.byref(h)) == ks.KS_EINVAL, args
    # a null handle is refused by every call
    assert ks.raw_call("ks_keyswitch", None, None, None, None, 1, None, None, None) == ks.KS_ENULL
    assert ks.raw_call("ks_ntt", None, None, 0, 1, 1, None) == ks.KS_ENULL
