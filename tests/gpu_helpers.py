"""Helpers shared by the GPU parity tests (moving seeded problems to the device,
error measures).  The oracle and the device library are only ever compared
here; neither imports the other."""
import numpy as np
import torch

import paper_2509_23018_amd as gw

FP64_TOL = 1e-12   # relative Frobenius bound for every FP64 result


def rel_fro(x, y) -> float:
    x = np.asarray(x)
    y = np.asarray(y)
    den = np.linalg.norm(y.reshape(-1))
    return float(np.linalg.norm((x - y).reshape(-1)) / (den if den > 0 else 1.0))


def device():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda", 0)


def to_dev(p, dev=None) -> gw.Chi0Problem:
    dev = dev or device()
    return gw.Chi0Problem(
        n=p.n, volume=p.volume,
        psi_v=torch.from_numpy(np.ascontiguousarray(p.psi_v)).to(dev),
        psi_c=torch.from_numpy(np.ascontiguousarray(p.psi_c)).to(dev),
        e_v=torch.from_numpy(np.ascontiguousarray(p.e_v)).to(dev),
        e_c=torch.from_numpy(np.ascontiguousarray(p.e_c)).to(dev),
        gvec=p.gvec, z=p.z)


def run_chi0(p, **kw) -> np.ndarray:
    dp = to_dev(p)
    kw.setdefault("pair_chunk", p.pair_chunk)
    kw.setdefault("spin", p.spin)
    chi = gw.gw_chi0(dp, **kw)
    torch.cuda.synchronize()
    return chi.cpu().numpy()
