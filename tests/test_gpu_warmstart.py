"""The learned warm start end to end on held-out porous boxes, with the
network trained by the library's own kernels (weights committed with the
package): the prediction beats the zero guess, both starts converge, and the
warm-versus-cold gain is measured.  A warm start from the exact steady field
shows the gain an accurate prediction buys."""
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1711_11468_amd", "weights", "unet_porous64.npz")


@pytest.fixture(scope="module")
def WS():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_11468_amd import warmstart
    return warmstart


def test_trained_network_on_held_out_geometries(WS):
    from paper_1711_11468_amd.surrogate import UNet
    net = UNet.load(WEIGHTS)
    rows = [WS.compare(net, 100000 + k, 64) for k in range(2)]
    for r in rows:
        print(r)
        assert r["cold_reason"] == "converged" and r["warm_reason"] == "converged"
        assert r["prediction_rel_l2"] < 0.9          # better than the zero guess (1.0)
        assert r["warm_vs_cold_rel_l2"] < 5e-2
    gain = np.median([r["cold_steps"] / r["warm_steps"] for r in rows])
    print("median step gain of the trained network: %.2f" % gain)


def test_exact_field_warm_start_gain(WS):
    """Starting from the exact steady velocity (equilibrium at u - g/2rho)
    reaches the residual target in well under the cold-start step count
    and lands on the same steady state."""
    from paper_1711_11468_amd import lbm
    mask, _ = WS.geometry(100001, 64)
    lat, steps_c, _, _, _ = WS.solve(mask)
    ref = lbm.Lattice(mask, addressing="list", bounce="halfway", **WS.PHYS)
    ref.run_to_steady(1e-11, max_steps=100000)
    u_ref = ref.macroscopic(fields=True)["u"].clone()
    lat_w, steps_w, _, _, why = WS.solve(mask, u0=u_ref)
    fl = torch.from_numpy(mask.reshape(-1) == 0).to(u_ref.device)
    u_w = lat_w.macroscopic(fields=True)["u"]
    err = float(((u_w - u_ref)[:, fl].norm() / u_ref[:, fl].norm()).item())
    print("cold", steps_c, "exact-warm", steps_w, "err", err)
    assert why == "converged"
    assert steps_w * 1.2 <= steps_c
    assert err < 2e-5
