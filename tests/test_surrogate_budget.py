"""Host checks of the surrogate rollout's gas-volume budget (CPU tensors):
the defect of a jump that moves exactly the inflow budget into the domain is
zero, the sign of the flux terms (gas entering through row 0 and leaving
through the last row) is fixed by hand-built fields, and `conserve` brings a
perturbed prediction onto the budget without touching the rows the flux
estimate reads or the other field planes.  The defect here is the FP64
reference (oracle/cno.py, volume_defect); the GPU kernel that the rollout
calls is compared with it in tests/test_gpu_surrogate.py."""
import numpy as np
import pytest
import torch

from oracle.cno import volume_defect
from paper_2409_10399_amd.surrogate_study import conserve


def defect(f0, f1, jump, chi):
    return volume_defect(f0.numpy(), f1.numpy(), jump, chi.numpy())


pytestmark = pytest.mark.filterwarnings("ignore")


def _fields(n=2, ny=24, nx=16, seed=0):
    g = torch.Generator().manual_seed(seed)
    f = torch.zeros((n, 6, ny, nx), dtype=torch.float64)
    f[:, 0] = 0.05 + 0.02 * torch.rand((n, ny, nx), generator=g, dtype=torch.float64)
    f[:, 1:5] = 1e-3 * torch.randn((n, 4, ny, nx), generator=g, dtype=torch.float64)
    f[:, 5] = 1e-4 * torch.randn((n, ny, nx), generator=g, dtype=torch.float64)
    return f


def test_defect_zero_for_a_jump_that_moves_the_budget():
    jump = 100
    chi = torch.tensor([0.0, 0.0], dtype=torch.float64)
    f0 = _fields()
    ny, nx = f0.shape[-2:]
    f0[:, 0, 0, :], f0[:, 2, 0, :] = 0.1, 0.01     # inlet row: alpha 0.1 moving +y at 0.01
    f0[:, 0, -1, :], f0[:, 2, -1, :] = 0.05, 0.01  # outlet row: alpha 0.05 leaving at 0.01
    inflow = nx * (0.1 * 0.01 - 0.05 * 0.01)       # per step, both ends
    f1 = f0.clone()
    f1[:, 0, 2:-2, :] += jump * inflow / ((ny - 4) * nx)
    assert np.all(defect(f0, f1, jump, chi) < 1e-12)
    # the same change with the flux reversed is a defect of twice the budget
    f1r = f0.clone()
    f1r[:, 0, 2:-2, :] -= jump * inflow / ((ny - 4) * nx)
    vol0 = f0[:, 0].sum(dim=(1, 2)).numpy()
    assert np.allclose(defect(f0, f1r, jump, chi), 2 * jump * inflow / vol0, rtol=1e-12)


def test_defect_counts_the_diffusive_flux():
    # alpha rising into the domain at the inlet (row 1 > row 0) with no
    # velocity: diffusion carries gas out through the inlet face
    jump, c = 100, 0.05
    chi = torch.tensor([c, c], dtype=torch.float64)
    f0 = _fields()
    ny, nx = f0.shape[-2:]
    f0[:, 2] = 0.0
    f0[:, 0, 0, :], f0[:, 0, 1, :] = 0.05, 0.07
    f0[:, 0, -2, :], f0[:, 0, -1, :] = 0.06, 0.06
    outflow = c * nx * 0.02
    f1 = f0.clone()
    f1[:, 0, 2:-2, :] -= jump * outflow / ((ny - 4) * nx)
    assert np.all(defect(f0, f1, jump, chi) < 1e-12)


def test_conserve_puts_a_prediction_on_the_budget():
    jump = 100
    chi = torch.tensor([0.02, 0.1], dtype=torch.float64)
    f0 = _fields(seed=1)
    f1 = f0 + 2e-3 * torch.randn(f0.shape, generator=torch.Generator().manual_seed(2), dtype=torch.float64)
    f1[:, 0].clamp_(min=0.0)
    before = defect(f0, f1, jump, chi)
    assert np.all(before > 1e-4)
    g = f1.clone()
    conserve(f0, g, jump, chi)
    assert np.all(defect(f0, g, jump, chi) < 1e-12)
    for rows in (slice(0, 2), slice(-2, None)):
        assert torch.equal(g[:, 0, rows], f1[:, 0, rows])
    assert torch.equal(g[:, 1:], f1[:, 1:])
    assert float(g[:, 0].min()) >= 0.0
    # the interior is scaled, not shifted: ratios between nodes stay
    ratio = g[:, 0, 2:-2] / f1[:, 0, 2:-2]
    assert torch.allclose(ratio, ratio[:, :1, :1].expand_as(ratio), rtol=1e-12)
