"""What training buys: the learned coarse solver trained by the GPU's own
forward/backward kernels beats the same solver with the untrained network
(z = 0, i.e. the base coefficients alone) against the coarsened fine
reference on held-out seeds.  Reduced scale: 512^2 fine runs, 8x coarsening
to 64^2, 8 training trajectories."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_training_gain_on_held_out_seeds():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2602_08670_amd import fv
    from paper_2602_08670_amd import learned_solver as LS

    n_fine, factor = 512, 8
    data = LS.dataset(range(100, 108), n_fine, factor, 96)
    print(f"[gain] data {tuple(data.shape)}", flush=True)
    model, hist, wall = LS.train(data, 300, B=16, T_max=4, lr=1e-3, n_fine=n_fine, factor=factor, log_every=100)
    print(f"[gain] training {wall:.1f} s, loss {hist[0][2]:.3e} -> {hist[-1][2]:.3e}", flush=True)
    res = LS.evaluate(model, [900, 901], n_fine, factor, 100, plain_sizes=(64,), chunk=50)
    base = LS.evaluate(fv.Model(LS.init_params(0), model.desc), [900, 901], n_fine, factor, 100, plain_sizes=(),
                       chunk=50)
    tr, un, pl = (res["cases"]["learned"]["rel_l2_h"], base["cases"]["learned"]["rel_l2_h"],
                  res["cases"]["plain64"]["rel_l2_h"])
    print(f"[gain] rel L2(h) vs reference: trained {tr:.3e}, untrained {un:.3e}, plain MINMOD {pl:.3e}", flush=True)
    assert tr < 0.9 * un
