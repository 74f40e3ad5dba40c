"""What training buys: the learned coarse solver trained by the GPU's own
forward/backward kernels beats the same solver with the untrained network
(z = 0, i.e. the base coefficients alone) against the coarsened fine
reference on held-out seeds.  Reduced scale: 512^2 fine runs, 8x coarsening
to 64^2, 8 training trajectories.

The claim is about the distribution over training runs, so the test trains
with five seeds and compares the median.  A short Adam run at a loss of
~1e-8 is chaotic in the rounding of its gradients (many components are
near zero, where Adam's normalised step follows their sign): two builds
whose gradients agree to 1e-5 relative in every layer end on different
iterates after a few iterations, and about one short run in ten ends on
parameters that are accurate over the T <= 4 training windows but drift
over the 100-step held-out rollout (rel L2(h) 5e-4 to 4e-2 where the others
reach about 2e-5)."""
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
    trained = []
    for seed in range(5):
        model, hist, wall = LS.train(data, 300, B=16, T_max=4, lr=1e-3, seed=seed, n_fine=n_fine, factor=factor)
        res = LS.evaluate(model, [900, 901], n_fine, factor, 100, plain_sizes=(64,), chunk=50)
        trained.append(res["cases"]["learned"]["rel_l2_h"])
        print(f"[gain] seed {seed}: training {wall:.1f} s, loss {hist[0][2]:.3e} -> {hist[-1][2]:.3e}, "
              f"held-out rel L2(h) {trained[-1]:.3e}", flush=True)
    # the untrained network outputs z = 0 whatever its (zero) last layer's inputs: the base coefficients
    base = LS.evaluate(fv.Model(LS.init_params(0), model.desc), [900, 901], n_fine, factor, 100, plain_sizes=(),
                       chunk=50)
    un, pl = base["cases"]["learned"]["rel_l2_h"], res["cases"]["plain64"]["rel_l2_h"]
    med = sorted(trained)[2]
    print(f"[gain] rel L2(h) vs reference: trained median {med:.3e}, untrained {un:.3e}, plain MINMOD {pl:.3e}",
          flush=True)
    assert med < 0.9 * un
