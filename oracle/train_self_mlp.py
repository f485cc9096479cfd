"""Train the learned self-collision network (Eq. 13, jointNERF form) on the
sphere model's signed closest link distance, as the paper trains its network
on distances between the robot's links (its own weights are not available).

Labels come from the oracle (oracle_self_distance, FP64); the network is
fitted with PyTorch on the CPU and its parameters are rounded to FP16-exact
values (the kernel's operand precision) and written in the flat layout of
inputs.SELF_MLP_LAYOUT to paper_2104_13542_amd/data/self_mlp_panda.npy.

    python -m oracle.train_self_mlp [--samples 200000] [--epochs 40]
"""
import argparse
import os

import numpy as np

import oracle
from paper_2104_13542_amd import inputs

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2104_13542_amd", "data",
                   "self_mlp_panda.npy")


def labelled_samples(n, seed):
    """Joint configurations uniform within the limits, with the sphere
    model's signed distance of each."""
    prob = inputs.config_self_mlp(0, n_particles=8, horizon=4)
    o = oracle.Oracle(prob)
    rng = np.random.default_rng(seed)
    q = rng.uniform(inputs.PANDA_Q_MIN, inputs.PANDA_Q_MAX, size=(n, 7))
    d = np.array([o.self_distance(qi) for qi in q])
    return q, d


def train(samples=200000, epochs=40, seed=0):
    import torch

    torch.manual_seed(seed)
    q, d = labelled_samples(samples, seed)
    x = torch.tensor(np.concatenate([np.sin(q), np.cos(q)], axis=1), dtype=torch.float32)
    y = torch.tensor(d, dtype=torch.float32)
    net = torch.nn.Sequential(torch.nn.Linear(14, 256), torch.nn.ReLU(), torch.nn.Linear(256, 128), torch.nn.ReLU(),
                              torch.nn.Linear(128, 64), torch.nn.ReLU(), torch.nn.Linear(64, 1))
    opt = torch.optim.Adam(net.parameters(), lr=1e-3)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, epochs)
    n = x.shape[0]
    for ep in range(epochs):
        perm = torch.randperm(n)
        tot = 0.0
        for k in range(0, n, 1024):
            idx = perm[k:k + 1024]
            loss = torch.nn.functional.smooth_l1_loss(net(x[idx]).squeeze(1), y[idx], beta=0.01)
            opt.zero_grad()
            loss.backward()
            opt.step()
            tot += loss.item() * idx.numel()
        sched.step()
        print("epoch %d loss %.5f" % (ep, tot / n), flush=True)
    W = [m for m in net if isinstance(m, torch.nn.Linear)]
    flat = np.concatenate([W[0].weight.detach().numpy().reshape(-1), W[0].bias.detach().numpy(),
                           W[1].weight.detach().numpy().reshape(-1), W[1].bias.detach().numpy(),
                           W[2].weight.detach().numpy().reshape(-1), W[2].bias.detach().numpy(),
                           W[3].weight.detach().numpy().reshape(-1), W[3].bias.detach().numpy()])
    assert flat.size == inputs.SELF_MLP_SIZE
    return flat.astype(np.float16).astype(np.float64)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=200000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args()
    prm = train(a.samples, a.epochs, a.seed)
    np.save(OUT, prm.astype(np.float32))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
