"""The allocation-free exact-sum entry point (fmm_direct_sampled_noalloc)
through the C-ABI: the same bits as fmm_direct_sampled, on two calls in a
row (the second smaller, so the static scratch holds the first call's
partial sums when it starts), and the size limit refused before any device
work."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1206_0115_amd import fmm, inputs


def noalloc(pos, q, idx):
    n, nt = pos.shape[0], idx.shape[0]
    phi = torch.empty(nt, dtype=torch.float64, device="cuda")
    f = torch.empty(nt, 3, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream()
    rc = fmm.lib().fmm_direct_sampled_noalloc(
        ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(q.data_ptr()), n,
        ctypes.c_void_p(idx.data_ptr()), nt, fmm.FMM_KERNEL_INV_R,
        ctypes.c_void_p(phi.data_ptr()), ctypes.c_void_p(f.data_ptr()),
        ctypes.c_void_p(int(s.cuda_stream)))
    assert rc == fmm.FMM_OK, fmm.last_error()
    s.synchronize()
    return phi.cpu().numpy(), f.cpu().numpy()


def test_limit_refused_without_device_work():
    lib = fmm.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the check comes first
    rc = lib.fmm_direct_sampled_noalloc(fake, fake, 10, fake, 262_145, 1, fake, fake, None)
    assert rc == fmm.FMM_ERR_ARG and "scratch" in fmm.last_error()
    assert lib.fmm_direct_sampled_noalloc(None, fake, 10, fake, 4, 1, fake, fake,
                                          None) == fmm.FMM_ERR_ARG


@pytest.mark.gpu
def test_noalloc_matches_allocating_entry_point():
    for n, nt, seed in ((400_000, 1000, 81), (30_000, 70, 82)):
        print(f"noalloc n={n} nt={nt}", flush=True)
        pos, q = inputs.uniform_cube(n, seed)
        pos_d, q_d = torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda()
        idx = torch.from_numpy(
            np.random.default_rng(seed).choice(n, nt, replace=False).astype(np.int64)).cuda()
        ref_phi, ref_f = fmm.direct_sampled(pos_d, q_d, idx)
        phi, f = noalloc(pos_d, q_d, idx)
        assert np.array_equal(phi, ref_phi.cpu().numpy())
        assert np.array_equal(f, ref_f.cpu().numpy())
