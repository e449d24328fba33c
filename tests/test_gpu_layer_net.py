"""The learned two-layer network of Sec. 5.5 on synthetic stand-ins: the
model of eq. (exp_model) with s = 2, A = I and lam = 5,
    E(U) = 1/2 ||U - f||^2 + lam R_area(U),
minimised by (i) the plain WMC iteration run for 1000 steps and (ii) a
two-layer HalfWindowNet (K learned kernels per layer, min-|.| activation)
trained by Adam to minimise E directly (unsupervised, as the paper's energy
table).  The paper trains on 10,000 BSDS500 patches, which are not
available; here 256 synthetic 128 x 128 patches (noise sigma 0.1, seeds
5000..5255) train and 64 others (seeds 6000..6063) evaluate.  Its printed
energies are therefore not comparable; the test checks the mechanism
(training lowers the energy below the untrained network's and below E(f))
and the paper's ordering against the 1000-step iteration."""
import numpy as np
import pytest
import torch

import oracle
import wmc_synth

pytestmark = pytest.mark.gpu

LAM = 5.0


def energy(u, f):
    """eq. (exp_model), s = 2, R_area with forward differences (zero at the
    last row / column), summed per image, averaged over the batch."""
    ux = torch.zeros_like(u)
    uy = torch.zeros_like(u)
    ux[..., :, :-1] = u[..., :, 1:] - u[..., :, :-1]
    uy[..., :-1, :] = u[..., 1:, :] - u[..., :-1, :]
    e = 0.5 * (u - f) ** 2 + LAM * torch.sqrt(1.0 + ux * ux + uy * uy)
    return e.sum(dim=(-2, -1)).mean()


def patches(seed0, n):
    return np.stack([wmc_synth.image(128, 128, 1, 0.1, seed=seed0 + i)[0][0] for i in range(n)])


def test_energy_matches_oracle():
    rng = np.random.default_rng(3)
    u = rng.uniform(0, 1, size=(13, 17))
    f = rng.uniform(0, 1, size=(13, 17))
    e = energy(torch.from_numpy(u), torch.from_numpy(f)).item()
    assert abs(e - oracle.energy_area(u, f, LAM)) <= 1e-9 * abs(e)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("K", [4, 8, 16])
def test_two_layer_network_energy(K):
    import paper_1903_07189_amd as W
    dev = "cuda:0"
    train = torch.from_numpy(patches(5000, 256)).to(dev)
    test = torch.from_numpy(patches(6000, 64)).to(dev)
    gen = torch.Generator().manual_seed(K)
    net = W.nn.HalfWindowNet(layers=2, K=K, lam=LAM, generator=gen, device=dev)
    with torch.no_grad():
        e_init = energy(net(test), test).item()
        e_f = energy(test, test).item()
        e_iter = energy(W.solve(test, LAM, 1000), test).item()
    opt = torch.optim.Adam(net.parameters(), lr=0.01)
    order = torch.randperm(256, generator=torch.Generator().manual_seed(1))
    for step in range(300):
        idx = order[(step * 32) % 256:(step * 32) % 256 + 32].to(dev)
        f = train[idx]
        loss = energy(net(f), f)
        opt.zero_grad()
        loss.backward()
        opt.step()
    with torch.no_grad():
        e_net = energy(net(test), test).item()
    print(f"\nK={K}: E(f) {e_f:.1f}, 2-layer untrained {e_init:.1f}, trained {e_net:.1f}, "
          f"iteration x1000 {e_iter:.1f}")
    assert e_net < e_init < e_f
    # the paper's observation (its energy table): two trained layers reach a
    # lower energy than 1000 plain iterations (measured here: 82040 vs 82203,
    # against a floor of lam * 128^2 = 81920 for a constant image)
    assert e_net < e_iter
