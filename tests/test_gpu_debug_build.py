"""The debug build libks_debug.so (the same kernels, every call first checking
that its inputs are canonical residues): KS_EINVAL before any work when a word
of an input is not below its limb's prime, the release library's output
otherwise. Rows a call does not read (a level handle's unused key rows) are
not checked."""
import ctypes
import os

import numpy as np
import pytest
import torch

from synth import ciphertext_batch, uniform_key, uniform_residues

from gpu_util import dev, empty, host

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_vp, _i = ctypes.c_void_p, ctypes.c_int


@pytest.fixture(scope="module")
def ks():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2603_16692_amd as k
    return k


@pytest.fixture(scope="module")
def dbg():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2603_16692_amd", "libks_debug.so"))
    lib.ks_params_create.argtypes = [_i, _i, _i, ctypes.POINTER(_vp)]
    lib.ks_params_at_level.argtypes = [_vp, _i, ctypes.POINTER(_vp)]
    lib.ks_params_destroy.argtypes = [_vp]
    lib.ks_params_destroy.restype = None
    lib.ks_keyswitch.argtypes = [_vp, _vp, _vp, _vp, _i, _vp, _vp, _vp]
    lib.ks_hrot.argtypes = [_vp, _vp, _i, _vp, _vp, _i, _vp, _vp, _vp]
    lib.ks_ntt.argtypes = [_vp, _vp, _i, _i, _i, _vp]
    lib.ks_bconv.argtypes = [_vp, _vp, _i, _vp, _i, _vp]
    lib.ks_moddown.argtypes = [_vp, _vp, _vp, _i, _vp, _vp]
    lib.ks_keymult.argtypes = [_vp, _vp, _vp, _vp, _i, _vp]
    return lib


def P(t):
    return ctypes.c_void_p(t.data_ptr())


def handle(dbg, *args):
    h = _vp()
    assert dbg.ks_params_create(*args, ctypes.byref(h)) == 0
    return h


def test_debug_build_rejects_non_canonical_inputs(ks, dbg):
    dnum, log_n, ell, batch = 2, 10, 5, 3
    G = ks.KsParams(dnum, log_n, ell)
    h = handle(dbg, dnum, log_n, ell)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    try:
        d = dev(ciphertext_batch(G.moduli[:ell], G.n, batch, seed_base=3100))
        evk = dev(uniform_key(G.moduli, G.n, G.ndig, seed=3200))
        ws = G.workspace(batch)
        ref = empty((batch, 2, ell, G.n))
        G.keyswitch(d, evk, ref, batch, ws)
        out = empty((batch, 2, ell, G.n))
        assert dbg.ks_keyswitch(h, P(d), P(evk), P(out), batch, None, P(ws), s) == 0
        assert np.array_equal(host(out), host(ref))
        # one word of d equal to its prime: refused, and out left as it was
        bad = d.clone()
        bad[1, 2, 17] = G.moduli[2]
        out.fill_(-7)
        assert dbg.ks_keyswitch(h, P(bad), P(evk), P(out), batch, None, P(ws), s) == ks.KS_EINVAL
        assert bool((out == -7).all())
        # a key word of a P row (digit 1, component 1, p_2) above its prime
        badk = evk.clone()
        badk[1, 1, ell + 2, 5] = G.moduli[ell + 2] + 3
        assert dbg.ks_keyswitch(h, P(d), P(badk), P(out), batch, None, P(ws), s) == ks.KS_EINVAL
        # HROT reads both components of its ciphertext
        ct = dev(ciphertext_batch(G.moduli[:ell], G.n, 2 * batch, seed_base=3300)).view(batch, 2, ell, G.n)
        ews = G.eval_workspace(batch)
        assert dbg.ks_hrot(h, P(ct), 5, P(evk), P(out), batch, None, P(ews), s) == 0
        ct[2, 1, 0, 0] = -1  # 2^64 - 1 as a residue
        assert dbg.ks_hrot(h, P(ct), 5, P(evk), P(out), batch, None, P(ews), s) == ks.KS_EINVAL
        # the step calls check the limbs they read: the NTT of the P limbs, BConv from digit 1, ModDown's acc
        x = dev(np.stack([uniform_residues(3400 + b, G.moduli[ell:], G.n) for b in range(batch)]))
        assert dbg.ks_ntt(h, P(x), ell, G.k, batch, s) == 0
        x[0, 1, 3] = G.moduli[ell + 1]
        assert dbg.ks_ntt(h, P(x), ell, G.k, batch, s) == ks.KS_EINVAL
        lo = G.alpha
        src = dev(np.stack([uniform_residues(3500 + b, G.moduli[lo:ell], G.n) for b in range(batch)]))
        dst = empty((batch, G.nl - (ell - lo), G.n))
        assert dbg.ks_bconv(h, P(src), 1, P(dst), batch, s) == 0
        src[2, 0, 9] = G.moduli[lo]
        assert dbg.ks_bconv(h, P(src), 1, P(dst), batch, s) == ks.KS_EINVAL
        acc = dev(np.stack([np.concatenate([uniform_residues(3600 + 2 * b + c, G.moduli, G.n) for c in range(2)])
                            for b in range(batch)]))
        mws = G.workspace(batch, ks.make_plan(ks.STAGED))
        assert dbg.ks_moddown(h, P(acc), P(out), batch, P(mws), s) == 0
        acc[1, G.nl + 3, 1] = G.moduli[3] + 1  # component 1, limb 3
        assert dbg.ks_moddown(h, P(acc), P(out), batch, P(mws), s) == ks.KS_EINVAL
        ext = dev(np.stack([np.concatenate([uniform_residues(3700 + 4 * b + j, G.moduli, G.n) for j in range(G.ndig)])
                            for b in range(batch)]))
        accd = empty((batch, 2, G.nl, G.n))
        assert dbg.ks_keymult(h, P(ext), P(evk), P(accd), batch, s) == 0
        ext[0, G.nl + ell, 0] = G.moduli[ell]  # digit 1, first P limb
        assert dbg.ks_keymult(h, P(ext), P(evk), P(accd), batch, s) == ks.KS_EINVAL
        torch.cuda.synchronize()
    finally:
        dbg.ks_params_destroy(h)


def test_debug_build_skips_rows_a_level_does_not_read(ks, dbg):
    dnum, log_n, ell, level, batch = 2, 10, 8, 3, 2
    top = ks.KsParams(dnum, log_n, ell)
    G = top.at_level(level)
    h = handle(dbg, dnum, log_n, ell)
    hl = _vp()
    assert dbg.ks_params_at_level(h, level, ctypes.byref(hl)) == 0
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    try:
        d = dev(ciphertext_batch(G.moduli[:level], G.n, batch, seed_base=3800))
        evk = dev(uniform_key(top.moduli, top.n, top.ndig, seed=3900))
        # rows of Q limbs the level does not have (and the top's second digit) are not read
        evk[0, 0, level + 1, :] = -1
        evk[1, 0, 0, :] = -1
        ws = G.workspace(batch)
        ref = empty((batch, 2, level, G.n))
        G.keyswitch(d, evk, ref, batch, ws)
        out = empty((batch, 2, level, G.n))
        assert dbg.ks_keyswitch(hl, P(d), P(evk), P(out), batch, None, P(ws), s) == 0
        assert np.array_equal(host(out), host(ref))
        evk[0, 1, level - 1, 4] = -1  # a row the level reads
        assert dbg.ks_keyswitch(hl, P(d), P(evk), P(out), batch, None, P(ws), s) == ks.KS_EINVAL
        torch.cuda.synchronize()
    finally:
        dbg.ks_params_destroy(hl)
        dbg.ks_params_destroy(h)
