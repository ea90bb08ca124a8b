"""Train the learned prior's UNet on the GPU with the library's own forward,
backward and Adam kernels (Sec. 4.2: supervised l1 loss, Adam, lr 1e-4,
batch 10, 128 x 128 patches).

Training pairs: seeded random-ellipse phantoms (clean) and copies with
independent Gaussian noise of standard deviation sigma ~ U(sigma_lo,
sigma_hi) on the real and imaginary parts; the network is conditioned on
sigma.  One epoch visits every phantom once (a random 128 x 128 crop each).
torch only holds the phantom set, cuts the crops and draws the noise.

    python -m paper_2411_01955_amd.train_unet --out weights.npz --epochs 100

Checkpoints (npz): FP32 parameters in the library layout, Adam moments,
step and epoch counters; ``--resume`` continues from one.
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import synth  # noqa: E402


def _phantom(args):
    n, seed = args
    return synth.phantom2d(n, seed)[0]


def make_phantoms(count, n, seed0, workers=8):
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return np.stack(list(ex.map(_phantom, [(n, seed0 + i) for i in range(count)], chunksize=16)))


def init_params(seed):
    """He-normal weights (last layer scaled by 0.1), zero biases, in the
    library's flat layout."""
    import paper_2411_01955_amd as pnp
    shapes = {l["name"]: ((l["cout"], l["taps"], l["cin"]), (l["cout"],)) for l in pnp.unet_layers()}
    return pnp.pack_unet_params(synth.he_normal(shapes, seed, last_scale={"out": 0.1}))


def save(path, net, epoch, args):
    np.savez(path, params=net.get("params").cpu().numpy(), adam_m=net.get("adam_m").cpu().numpy(),
             adam_v=net.get("adam_v").cpu().numpy(), step=net.step, epoch=epoch,
             config=np.array(str(vars(args))))


def load_weights(path):
    """FP32 parameters (library layout) of a checkpoint or weights file."""
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float32)


def psnr(x, ref):
    import torch
    mse = torch.mean(torch.abs(x - ref) ** 2).item()
    peak = torch.max(torch.abs(ref)).item()
    return 10 * math.log10(peak * peak / max(mse, 1e-30))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--phantoms", type=int, default=2000)
    ap.add_argument("--size", type=int, default=320)
    ap.add_argument("--patch", type=int, default=128)
    ap.add_argument("--batch", type=int, default=10)
    ap.add_argument("--epochs", type=int, default=100)
    ap.add_argument("--lr", type=float, default=1e-4)
    ap.add_argument("--sigma-lo", type=float, default=0.001)
    ap.add_argument("--sigma-hi", type=float, default=0.1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-minutes", type=float, default=0.0, help="stop (and save) after this long")
    ap.add_argument("--resume", default=None)
    ap.add_argument("--log-every", type=int, default=100)
    args = ap.parse_args(argv)

    import torch
    import paper_2411_01955_amd as pnp
    t0 = time.time()
    dev = torch.device("cuda")
    clean = torch.from_numpy(make_phantoms(args.phantoms, args.size, synth.SEED_TRAIN)).to(dev)
    held = torch.from_numpy(make_phantoms(4, args.size, synth.SEED_HELDOUT)).to(dev)
    print(f"[train] {args.phantoms} phantoms {args.size}^2 ready in {time.time() - t0:.1f}s", flush=True)

    if args.resume:
        with np.load(args.resume, allow_pickle=False) as z:
            net = pnp.UNet(z["params"].astype(np.float32))
            net.set("adam_m", z["adam_m"].astype(np.float32))
            net.set("adam_v", z["adam_v"].astype(np.float32))
            net.step = int(z["step"])
            epoch0 = int(z["epoch"])
    else:
        net = pnp.UNet(init_params(args.seed))
        epoch0 = 0

    B, P, n = args.batch, args.patch, args.size
    gen = torch.Generator(device=dev)
    target = torch.empty((B, P, P), dtype=torch.complex64, device=dev)
    noisy = torch.empty_like(target)
    sig = torch.empty(B, dtype=torch.float32, device=dev)
    # validation: the held-out phantoms at three noise levels, full size
    vs = torch.tensor([0.01, 0.03, 0.1, 0.05], dtype=torch.float32, device=dev)
    vg = torch.Generator(device=dev)
    vg.manual_seed(12345)
    vnoise = (torch.randn(held.shape, generator=vg, device=dev) + 1j * torch.randn(held.shape, generator=vg, device=dev))
    vnoisy = (held + vs[:, None, None] * vnoise).to(torch.complex64).contiguous()

    def validate():
        d = net.forward(vnoisy, vs)
        return [(psnr(vnoisy[i], held[i]), psnr(d[i], held[i])) for i in range(held.shape[0])]

    steps_per_epoch = args.phantoms // B
    t_train = time.time()
    done = False
    epoch = epoch0
    for epoch in range(epoch0, args.epochs):
        rng = np.random.default_rng((args.seed, epoch))
        order = rng.permutation(args.phantoms)
        offs = rng.integers(0, n - P + 1, (args.phantoms, 2))
        gen.manual_seed(args.seed * 100003 + epoch)
        run = 0.0
        for it in range(steps_per_epoch):
            idx = order[it * B:(it + 1) * B]
            for j, i in enumerate(idx):
                y0, x0 = offs[i]
                target[j] = clean[i, y0:y0 + P, x0:x0 + P]
            torch.rand(B, generator=gen, device=dev, out=sig)
            sig.mul_(args.sigma_hi - args.sigma_lo).add_(args.sigma_lo)
            nz = torch.randn((2, B, P, P), generator=gen, device=dev)
            torch.add(target, torch.complex(nz[0], nz[1]) * sig[:, None, None], out=noisy)
            net.forward(noisy, sig, train=True)
            loss = net.backward(noisy, target)
            net.adam_step(args.lr)
            if (it + 1) % args.log_every == 0:
                run = float(loss.item())
                el = time.time() - t_train
                print(f"[train] epoch {epoch + 1} step {net.step} loss {run:.4e} "
                      f"({el / max(1, net.step - epoch0 * steps_per_epoch):.4f} s/step, {el:.0f}s)", flush=True)
            if args.max_minutes and time.time() - t_train > 60 * args.max_minutes:
                done = True
                break
        v = validate()
        print(f"[train] epoch {epoch + 1} held-out PSNR noisy->denoised: " +
              ", ".join(f"{a:.1f}->{b:.1f}" for a, b in v), flush=True)
        save(args.out, net, epoch + 1 if not done else epoch, args)
        if done:
            break
    torch.cuda.synchronize()
    print(f"[train] finished: {net.step} steps in {time.time() - t_train:.1f}s, saved {args.out}", flush=True)


if __name__ == "__main__":
    main()
