"""A case read from OpenCFD-FWH files (Appendix A layouts, include/fwh_io.h)
runs through the HIP path exactly as the same arrays handed over directly:
bit-identical output, and parity with the FP64 oracle on the data as read
(relative L2 1e-11 for the FP64 form, 1e-5 for FP32).  The frames are read
into page-locked host tensors and copied to the device asynchronously."""
import numpy as np
import pytest

from gpu_common import oracle_forward, rel_l2, to_device, valid_mask
from paper_2312_16263_amd import fileio
from workloads import configs, surfaces

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-11, "f32": 1e-5}


def _case():
    x = np.array([[7.0, -3.0, 1.0], [-20.0, 2.0, 0.5], [0.0, 12.0, -4.0], [40.0, 0.0, 0.0], [0.1, -6.0, 2.0]])
    return configs.Case("dip_files", surfaces.sphere(1.0, 12, 24), x, 0.5, 10.0, 1 / 100, 300, tau0=0.0,
                        kind="dipole")


@pytest.mark.parametrize("fmt", [fileio.BINARY, fileio.ASCII])
@pytest.mark.parametrize("mode", ["f64", "f32"])
def test_case_from_files_matches_direct_arrays(tmp_path, fmt, mode):
    import torch
    c = _case()
    rho, u, pp = c.data()
    # three Faces over the 12 x 24 panel grid, one dimension 1 each
    dims = np.array([[6, 24, 1], [1, 3, 24], [3, 1, 24]], dtype=np.int64)
    geom = fileio.Geometry(dims, c.surface.y, c.surface.normal, c.surface.dS)
    d = str(tmp_path / "case")
    fileio.save_case(d, c.mach, c.aoa_deg, c.dtau / 5, 500, 5, geom, c.x_obs, rho, u, pp, fmt=fmt)
    print(f"[files -> HIP] fmt={fmt} mode={mode} P={c.n_panels} O={c.n_obs} N={c.n_tau}", flush=True)
    fc = fileio.load_case(d, dtype=mode, pinned=True, threads=4)
    assert fc.rho.is_pinned() and fc.u.is_pinned() and fc.pp.is_pinned()
    plan = fc.plan(mode)
    dev = [t.to("cuda", non_blocking=True) for t in (fc.rho, fc.u, fc.pp)]
    out_files = plan.forward(*dev).clone()
    tdt = torch.float64 if mode == "f64" else torch.float32
    direct = plan.forward(*to_device((rho, u, pp), tdt))
    torch.cuda.synchronize()
    assert torch.equal(out_files, direct)
    # frame 0 is solver step 500 at dt = dtau/5: tau0 = 1.0 shifts every window start by 1.0
    assert fc.tau0 == pytest.approx(1.0, rel=1e-15)
    # the oracle sees the data as stored (FP32 frames are the rounded doubles)
    p_ref, ts_ref, nt_ref = oracle_forward(c, *(t.numpy().astype(np.float64) for t in (fc.rho, fc.u, fc.pp)))
    np.testing.assert_allclose(plan.window.t_start, ts_ref + fc.tau0, rtol=1e-14, atol=0)
    assert np.array_equal(plan.window.n_t, nt_ref)
    p = out_files.double().cpu().numpy()
    m = valid_mask(nt_ref, p.shape[1])
    err = rel_l2(p, p_ref, m)
    print(f"    rel L2 vs oracle = {err:.3e} (tol {TOL[mode]:.0e})", flush=True)
    assert err <= TOL[mode], err


@pytest.mark.parametrize("fmt,block", [(fileio.BINARY, 7), (fileio.ASCII, 64)])
def test_frames_streamed_to_device(tmp_path, fmt, block):
    """Blocks of frames parsed into two page-locked buffers while the previous
    block is copied: the device tensors equal the host read, bit for bit
    (ragged last block with block = 7)."""
    import torch
    c = _case()
    rho, u, pp = c.data()
    dims = np.array([[6, 24, 1], [1, 3, 24], [3, 1, 24]], dtype=np.int64)
    geom = fileio.Geometry(dims, c.surface.y, c.surface.normal, c.surface.dS)
    d = str(tmp_path / "case")
    fileio.save_case(d, c.mach, c.aoa_deg, c.dtau, 0, 1, geom, c.x_obs, rho, u, pp, fmt=fmt)
    for dtype in ("f64", "f32"):
        fc = fileio.load_case(d, dtype=dtype, device="cuda", threads=3)
        torch.cuda.synchronize()
        ref = fileio.load_case(d, dtype=dtype)
        for dev_t, host in zip((fc.rho, fc.u, fc.pp), (ref.rho, ref.u, ref.pp)):
            assert dev_t.is_cuda
            np.testing.assert_array_equal(dev_t.cpu().numpy(), host)
        out = fileio.read_frames_to_device(d, 0, 1, c.n_tau, fmt, dims, dtype=dtype, block=block)
        np.testing.assert_array_equal(out[1].cpu().numpy(), ref.u)
