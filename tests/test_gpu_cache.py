"""The software-managed device cache on the GPU (device backend, pinned host buffers): the
library held to the plain model op by op with real bytes moved through host and device
views, and the hopping term applied to fields that live in host memory and share a device
budget smaller than the working set, bit for bit equal to applies on device-resident
fields."""

import ctypes
import random

import pytest
import torch

from oracle import cache_model as M
from synth import fields as F

from gpu_util import make, need_gpu, to_dev

pytestmark = pytest.mark.gpu
KB = 4096


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def D():
    from paper_2203_06777_amd import dwf

    return dwf


def _hip():
    h = ctypes.CDLL("libamdhip64.so")
    h.hipMemset.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t]
    h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return h


@pytest.mark.parametrize("seed", range(4))
def test_device_cache_matches_the_model(seed):
    hip = _hip()
    torch.cuda.synchronize()
    rng = random.Random(200 + seed)
    wm = rng.choice([2, 3]) * KB
    keys = [f"k{i}" for i in range(rng.choice([4, 6]))]
    bufs = {k: torch.zeros(KB, dtype=torch.uint8, pin_memory=True) for k in keys}
    m = M.CacheModel(wm)
    c = D().dwf_cache_create(wm, D().DWF_CACHE_DEVICE)
    last = {k: 0 for k in keys}
    scratch = ctypes.create_string_buffer(KB)
    for step in range(120):
        k, intent = rng.choice(keys), rng.randrange(4)
        m.open(k, KB, intent)
        view = D().dwf_cache_open(c, bufs[k], KB, intent)
        if intent in (M.ACC_READ, M.ACC_WRITE):
            torch.cuda.synchronize()
            assert hip.hipMemcpy(scratch, view, KB, 2) == 0  # device -> host
            got = scratch.raw
        else:
            assert view == bufs[k].data_ptr()
            got = bytes(bufs[k].numpy())
        assert got == bytes([last[k] % 251]) * KB, (step, k, intent)
        if intent in (M.ACC_WRITE, M.CPU_WRITE):
            last[k] += 1
            if intent == M.ACC_WRITE:
                assert hip.hipMemset(view, last[k] % 251, KB) == 0
            else:
                bufs[k].fill_(last[k] % 251)
        m.close(k)
        D().dwf_cache_close(c, bufs[k])
        snap, mc = m.snapshot()
        for kk, (s, r_, res) in snap.items():
            assert D().dwf_cache_query(c, bufs[kk]) == (s, r_, res), (step, kk)
        st = D().dwf_cache_get_stats(c)
        assert (st["h2d_count"], st["d2h_count"], st["evictions"], st["held_bytes"]) == mc
    D().dwf_cache_destroy(c)
    for k in keys:
        assert bytes(bufs[k].numpy()) == bytes([last[k] % 251]) * KB


def test_dhop_on_host_fields_through_the_cache():
    """Six input and six output fields of 8^4 x 8 (FP32) in pinned host memory, device budget
    of four fields: every apply evicts, dirty outputs are written back; the results equal
    applies on device-resident copies bit for bit, and the copy counts equal the model's."""
    dims, ls = (8, 8, 8, 8), 8
    op, u = make(dims, ls, seed_u=301)
    nb = op.field("f32").numel()  # bytes (fields are byte tensors)
    n = 6
    ins, outs, want = [], [], []
    for i in range(n):
        psi = F.fermion_cb(dims, ls, 302 + i)
        dev = op.pack(to_dev(psi), 0, "f32")
        w = op.zeros("f32")
        D().dwf_dhop(op.handle, w, dev, 1, i % 2, "f32")
        want.append(w)
        h = torch.empty(dev.numel(), dtype=dev.dtype, pin_memory=True)
        h.copy_(dev)
        ins.append(h)
        outs.append(torch.zeros(dev.numel(), dtype=dev.dtype, pin_memory=True))
    torch.cuda.synchronize()
    c = D().dwf_cache_create(4 * nb, D().DWF_CACHE_DEVICE)
    m = M.CacheModel(4 * nb)
    for rnd in range(2):
        for i in range(n):
            vi = D().dwf_cache_open(c, ins[i], nb, D().DWF_ACC_READ)
            vo = D().dwf_cache_open(c, outs[i], nb, D().DWF_ACC_WRITE)
            m.open(("in", i), nb, M.ACC_READ)
            m.open(("out", i), nb, M.ACC_WRITE)
            D().dwf_dhop(op.handle, vo, vi, 1, i % 2, "f32")
            D().dwf_cache_close(c, ins[i])
            D().dwf_cache_close(c, outs[i])
            m.close(("in", i))
            m.close(("out", i))
    st = D().dwf_cache_get_stats(c)
    assert (st["h2d_count"], st["d2h_count"], st["evictions"]) == (m.h2d, m.d2h, m.evictions)
    assert st["evictions"] > 0 and st["d2h_count"] > 0
    for i in range(n):
        h = D().dwf_cache_open(c, outs[i], nb, D().DWF_CPU_READ)
        assert h == outs[i].data_ptr()
        assert torch.equal(outs[i], want[i].cpu()), i
        D().dwf_cache_close(c, outs[i])
    D().dwf_cache_destroy(c)
    op.close()
