"""What training buys for the learned Euler discretisation: the network
trained by the GPU's own forward/adjoint/Adam kernels beats both the
untrained network (the base coefficients alone) and the plain MINMOD scheme
on the same coarse grid, against the coarsened fine reference on held-out
seeds.  Reduced scale: 256^2 fine periodic Euler runs coarsened 8x to 32^2,
24 training trajectories of 100 coarse steps, 1200 iterations with unrolls
of up to 16 steps, the iterate kept by four validation rollouts; four
held-out seeds, 100 coarse steps each, every one of them must win."""
import math

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_learned_euler_gain_on_held_out_seeds():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2602_08670_amd import fv
    from paper_2602_08670_amd import learned_euler_solver as LE
    from paper_2602_08670_amd.learned_solver import rel_l2

    n_fine, factor, steps = 256, 8, 100
    n = n_fine // factor
    dt_c = LE.fine_dt(n_fine) * factor
    data = torch.stack([LE.trajectory(s, n_fine, factor, steps) for s in range(300, 324)])
    print(f"[euler gain] data {tuple(data.shape)}", flush=True)

    def refs_of(seeds):
        q0, ref = [], []
        for s in seeds:
            tr = LE.trajectory(s, n_fine, factor, steps)
            q0.append(tr[0].cpu().numpy())
            ref.append(tr[-1].double().cpu().numpy())
        return q0, ref

    vq, vr = refs_of([700, 701, 702, 703])
    tq, tr_ = refs_of([900, 901, 902, 903])
    mean, inv_std, std = LE.normalisation(data)
    p0 = LE.init_params(0)
    B, T_max, iters, lr, lr_final = 16, 16, 1200, 1e-3, 2e-5
    net = fv.EulerLearned(p0, B, n, n, dt_c, mean=mean, inv_std=inv_std)
    vnet = fv.EulerLearned(p0, 4, n, n, dt_c, mean=mean, inv_std=inv_std)
    trn = fv.EulerTrainer(net, fv.make_euler_train_config(B, n, n, T_max, dt_c, scale=tuple(std), lr=lr))

    def score():
        vnet.params.copy_(net.params)
        return LE.rollout_score(vnet, vq, vr, steps)

    rng = np.random.default_rng(1)
    best = (score(), 0, net.params.clone())
    for it in range(iters):
        T = min(T_max, 1 + (it * T_max) // (iters // 2))
        ti = torch.as_tensor(rng.integers(0, data.shape[0], B), device="cuda")
        ki = torch.as_tensor(rng.integers(0, data.shape[1] - T, B), device="cuda")
        tg = data[ti[None, :], ki[None, :] + torch.arange(1, T + 1, device="cuda")[:, None]]
        trn.step(data[ti, ki], tg)
        trn.set_lr(lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * it / (iters - 1))))
        trn.adam()
        if (it + 1) % 100 == 0:
            sc = score()
            if sc < best[0]:
                best = (sc, it + 1, net.params.clone())
    trn.close()

    def rollout(params):
        e = fv.EulerLearned(params.cpu().numpy(), 4, n, n, dt_c, mean=mean, inv_std=inv_std)
        q = torch.tensor(np.stack(tq), device="cuda").contiguous()
        e.step(q, steps)
        fb, rd, fr, rc = e.stats()
        out = q.cpu().double().numpy()
        e.close()
        assert rc == fv.FV_OK
        return [rel_l2(out[b, 0], tr_[b][0]) for b in range(4)]

    got = rollout(best[2])
    base = rollout(torch.tensor(p0))
    plain = []
    for b in range(4):
        s = fv.Solver(tq[b], prec=fv.FV_F32, dt_fixed=dt_c)
        s.run(steps)
        plain.append(rel_l2(s.state()[0], tr_[b][0]))
        s.close()
    print(f"[euler gain] kept iteration {best[1]} (val {best[0]}); held-out rel L2(rho): trained "
          f"{[f'{x:.2e}' for x in got]}, untrained {[f'{x:.2e}' for x in base]}, "
          f"plain MINMOD {n}^2 {[f'{x:.2e}' for x in plain]}", flush=True)
    for g, b, p in zip(got, base, plain):
        assert g < 0.9 * b
        assert g < p
    net.close()
    vnet.close()
