"""The allocation-free emergent intensity (nlte_emergent_intensity_noalloc) against the
allocating entry point, through the C-ABI (GPU)."""
import ctypes as ct

import numpy as np
import pytest

from paper_1701_01607_amd import synth

pytestmark = pytest.mark.gpu


def test_noalloc_emergent_intensity_equals_the_allocating_entry_point():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    from paper_1701_01607_amd import nlte
    ctx = nlte.Context(0, torch.cuda.current_stream().cuda_stream)
    lib = ctx.lib
    mus = np.ascontiguousarray([[0.0, 0.0, 1.0], [0.3, -0.2, 0.93], [-0.5, 0.1, 0.4]], dtype=np.float64)
    mptr = mus.ctypes.data_as(ct.c_void_p)
    # a plane of 96x96 points holds 113 frequencies per scratch chunk, so the first call
    # (205 frequencies) runs two chunks; the second call is a smaller input in one chunk
    cases = [(96, 96, 9, 41, nlte.MIXED), (12, 10, 7, 9, nlte.FP64)]
    for nx, ny, nz, nfreq, prec in cases:
        print(f"case {nx}x{ny}x{nz} nfreq={nfreq} precision={prec}", flush=True)
        atom = synth.caii_like_atom(nfreq)
        atm = synth.atmos_stratified(nx=nx, ny=ny, nz=nz, dx=100 * synth.KM, seed=nx + nz)
        job = ctx.job(ctx.atmos(atm), ctx.atom(atom), nlte.SolveParams(method=nlte.MALI, precision=prec, nlev=1))
        job.mali(0, 2)
        nf = sum(len(l["q"]) for l in atom["lines"])
        out = torch.full((mus.shape[0], nf, ny, nx), float("nan"), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        ctx.check(lib.nlte_emergent_intensity_noalloc(ctx.h, job.id, mus.shape[0], mptr, ct.c_void_p(out.data_ptr())))
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0, "the allocation-free call changed free device memory"
        ref = torch.empty_like(out)
        ctx.check(lib.nlte_emergent_intensity(ctx.h, job.id, mus.shape[0], mptr, ct.c_void_p(ref.data_ptr()),
                                              nlte.MEM_DEVICE))
        torch.cuda.synchronize()
        assert torch.isfinite(ref).all()
        assert torch.equal(out, ref)
        # host output is rejected before any work
        host = np.empty((mus.shape[0], nf, ny, nx), dtype=np.float32)
        rc = lib.nlte_emergent_intensity_noalloc(ctx.h, job.id, mus.shape[0], mptr, host.ctypes.data_as(ct.c_void_p))
        assert rc == nlte.E_INVALID
        job.close()
    ctx.close()
