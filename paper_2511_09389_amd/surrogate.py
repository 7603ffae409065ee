"""Learned surrogate of the march, with the march as fallback.

Not part of the paper: a six-layer 3x3x3 convolutional network (32 channels, GELU,
residual blocks) that turns a cheap march (N_Omega / 8 rays) into an estimate of the full
march. Inputs per voxel: log kappa, j, and the cheap field (over its root-mean-square s,
and as a standardised log); output: a correction to the cheap field in units of s, so the
squared-error loss is the squared relative L2 error of the predicted field. Every step runs in the library's kernels: the cheap and the full march, the
input features, the bf16 matrix-core convolutions and their gradients, the loss, Adam and
the output transform; PyTorch only holds the buffers.

Fallback: the prediction is accepted when its relative L2 distance from the cheap field
is at most a threshold calibrated on validation samples (the largest value at which every
accepted validation prediction was within the error target of the full march); otherwise
the full march runs and its field is returned.
"""

import math
import time

import numpy as np
import torch

from . import inputs, rtmi

LAYERS = 6
C = rtmi.CONV_CHANNELS
CHEAP_DIVISOR = 8
N_FEATURES = 4


class SurrogateNet:
    """Weights (fp32 masters, bf16 copies) and Adam state of the network."""

    def __init__(self, device, seed=0, residual_scale=0.1):
        g = torch.Generator().manual_seed(seed)
        self.device = device
        self.w, self.b, self.wb = [], [], []
        for l in range(LAYERS):
            fan_in = 27 * (N_FEATURES if l == 0 else C)
            std = math.sqrt(2.0 / fan_in) * (residual_scale if 0 < l < LAYERS - 1 else 1.0)
            if l == LAYERS - 1:
                std = 1e-3                     # start near "no correction"
            w = torch.randn((27, C, C), generator=g) * std
            if l == 0:
                w[:, :, N_FEATURES:] = 0.0     # inputs beyond the features are zero
            if l == LAYERS - 1:
                w[:, 1:, :] = 0.0              # only channel 0 is read
            self.w.append(w.to(device).contiguous())
            self.b.append(torch.zeros(C, device=device))
            self.wb.append(self.w[-1].to(torch.bfloat16).contiguous())
        self.m = [torch.zeros_like(t) for t in self.w + self.b]
        self.v = [torch.zeros_like(t) for t in self.w + self.b]
        self.step = 0

    def forward(self, x, keep=False):
        """x: bf16 [n][d][h][w][32]. Returns (y, cache); cache holds each layer's input and,
        when keep, its fp32 pre-activation."""
        h, cache = x, []
        for l in range(LAYERS):
            z = torch.empty(x.shape, dtype=torch.float32, device=x.device) if keep and l < LAYERS - 1 else None
            if l == 0:
                y = rtmi.conv3d_forward(h, self.wb[l], bias=self.b[l], gelu=True, z=z)
            elif l < LAYERS - 1:
                y = rtmi.conv3d_forward(h, self.wb[l], bias=self.b[l], residual=h, gelu=True, z=z)
            else:
                y = rtmi.conv3d_forward(h, self.wb[l], bias=self.b[l], gelu=False)
            cache.append((h, z))
            h = y
        return h, cache

    def backward(self, cache, dz_last, dw=None, db=None):
        """Gradients (dW list, db list) of the loss whose dL/dy (channel 0) seeds dz_last,
        added into dw, db when given (accumulation over a batch)."""
        dw = [torch.zeros_like(w) for w in self.w] if dw is None else dw
        db = [torch.zeros_like(b) for b in self.b] if db is None else db
        dz, dh = dz_last, None
        for l in range(LAYERS - 1, -1, -1):
            h_in, _ = cache[l]
            rtmi.conv3d_backward_weight(h_in, dz, dw[l], db[l])
            if l == 0:
                break
            dh_prev = torch.empty(h_in.shape, dtype=torch.float32, device=h_in.device)
            dz_prev = torch.empty_like(h_in)
            rtmi.conv3d_backward_data(dz, self.wb[l], residual=dh if 0 < l < LAYERS - 1 else None,
                                      zprev=cache[l - 1][1], dh=dh_prev, dz_prev=dz_prev)
            dz, dh = dz_prev, dh_prev
        return dw, db

    def apply(self, dw, db, lr):
        self.step += 1
        params = self.w + self.b
        grads = dw + db
        for i, (p, g) in enumerate(zip(params, grads)):
            rtmi.adam_step(p, self.m[i], self.v[i], g, self.wb[i] if i < LAYERS else None, lr, self.step)

    def state(self):
        return {"w": [w.cpu() for w in self.w], "b": [b.cpu() for b in self.b]}

    def state_dict(self):
        """Weights, biases, both Adam moments and the step count (host tensors), enough to
        resume training exactly where it stopped."""
        return {"w": [w.detach().cpu() for w in self.w], "b": [b.detach().cpu() for b in self.b],
                "m": [t.detach().cpu() for t in self.m], "v": [t.detach().cpu() for t in self.v],
                "step": torch.tensor(self.step, dtype=torch.int64)}

    def load_state_dict(self, sd):
        def put(dst, src, name):
            if len(dst) != len(src):
                raise ValueError(f"checkpoint has {len(src)} {name} tensors, expected {len(dst)}")
            for d, t in zip(dst, src):
                if tuple(d.shape) != tuple(t.shape):
                    raise ValueError(f"checkpoint {name} shape {tuple(t.shape)} != {tuple(d.shape)}")
                d.copy_(t)
        put(self.w, sd["w"], "w")
        put(self.b, sd["b"], "b")
        put(self.m, sd["m"], "m")
        put(self.v, sd["v"], "v")
        self.step = int(sd["step"])
        for l in range(LAYERS):
            self.wb[l].copy_(self.w[l].to(torch.bfloat16))


def make_sample(seed, device, n=64, n_src=16, num_rays=4096, ds=0.5, c=64.0, dt=1.0,
                cheap_divisor=CHEAP_DIVISOR):
    """(j, kappa, cheap field, full field) of one seeded turbulent sample, on the device."""
    w = inputs.surrogate_sample(seed, n=n, n_src=n_src, num_rays=num_rays, ds=ds, c=c, dt=dt)
    j = torch.from_numpy(w.j_map).to(device)
    k = torch.from_numpy(w.kappa_map).to(device)
    full = rtmi.trace_multi(j, k, w.source_pos, w.num_rays, w.step_size, w.radiation_velocity, w.time_step)
    cheap = rtmi.trace_multi(j, k, w.source_pos, np.maximum(w.num_rays // cheap_divisor, 1), w.step_size,
                             w.radiation_velocity, w.time_step)
    return w, j, k, cheap, full


class Surrogate:
    """A trained network with its input statistics and calibrated acceptance threshold."""

    def __init__(self, net, stats, threshold=0.0, cheap_divisor=CHEAP_DIVISOR):
        self.net, self.stats, self.threshold = net, np.asarray(stats, np.float32), float(threshold)
        self.cheap_divisor = int(cheap_divisor)

    @property
    def floor(self):
        return float(self.stats[5])

    def save(self, path):
        """Checkpoint: the network's state_dict, the input statistics and the threshold."""
        torch.save({"net": self.net.state_dict(), "stats": torch.from_numpy(self.stats.copy()),
                    "threshold": torch.tensor(self.threshold, dtype=torch.float64),
                    "cheap_divisor": torch.tensor(self.cheap_divisor, dtype=torch.int64)}, path)

    @classmethod
    def load(cls, path, device):
        sd = torch.load(path, map_location="cpu", weights_only=True)
        net = SurrogateNet(device)
        net.load_state_dict(sd["net"])
        return cls(net, sd["stats"].numpy(), float(sd["threshold"]), int(sd.get("cheap_divisor", CHEAP_DIVISOR)))

    def features(self, j, k, cheap):
        """(x, scale_sums) of one sample."""
        return rtmi.surrogate_features(j, k, cheap, self.stats)

    @staticmethod
    def target(cheap, full, scale_sums):
        """Training target: (full - cheap) / s, s the cheap field's root-mean-square."""
        s = torch.sqrt(scale_sums[0] / cheap.numel())
        return ((full - cheap.clamp_min(0)) / s).contiguous()

    def predict(self, j, k, cheap):
        """(field, check): the network's field and its relative L2 distance from cheap."""
        x, sums = self.features(j, k, cheap)
        y, _ = self.net.forward(x)
        field, chk = rtmi.surrogate_output(y, cheap, sums)
        c = chk.cpu().numpy()
        return field, float(math.sqrt(c[0] / max(c[1], 1e-300)))

    def run(self, w, j, k):
        """Field of one problem: the surrogate when its check passes, else the full march.
        Returns (field, used_surrogate)."""
        cheap = rtmi.trace_multi(j, k, w.source_pos, np.maximum(w.num_rays // self.cheap_divisor, 1), w.step_size,
                                 w.radiation_velocity, w.time_step)
        field, check = self.predict(j, k, cheap)
        if check <= self.threshold:
            return field, True
        return rtmi.trace_multi(j, k, w.source_pos, w.num_rays, w.step_size, w.radiation_velocity,
                                w.time_step), False


def input_stats(samples):
    """Standardisation of the features from training samples [(w, j, k, cheap, full)]."""
    lk = np.concatenate([np.log(np.maximum(s[2].cpu().numpy().ravel(), 1e-30)) for s in samples])
    jm = max(float(s[1].max()) for s in samples)
    floor = 1e-6 * float(np.median([float(s[4].max()) for s in samples]))
    lc = np.concatenate([np.log(np.maximum(s[3].cpu().numpy().ravel(), 0) + floor) for s in samples])
    return np.array([lk.mean(), 1.0 / lk.std(), 1.0 / max(jm, 1e-30), lc.mean(), 1.0 / lc.std(), floor], np.float32)


def rel_l2(a, b):
    a, b = a.double(), b.double()
    return float((a - b).norm() / b.norm())


def learning_rate(lr, step, total, warmup, schedule):
    """Base rate lr after a linear warm-up of `warmup` steps, then constant, halved at every
    third of the run ("step"), or on a cosine to zero ("cosine")."""
    if warmup > 0 and step < warmup:
        return lr * (step + 1) / warmup
    if schedule == "cosine":
        frac = (step - warmup) / max(total - warmup, 1)
        return lr * 0.5 * (1.0 + math.cos(math.pi * min(frac, 1.0)))
    if schedule == "step":
        return lr * 0.5 ** (3 * step // max(total, 1))
    return lr


def train(train_samples, device, epochs=4, lr=2e-3, seed=0, log=None, batch=1, warmup=0, schedule="step",
          cheap_divisor=CHEAP_DIVISOR):
    """Train on [(w, j, k, cheap, full)] with Adam on the mean over `batch` samples of the
    loss (their weight gradients accumulate before each step); returns (Surrogate, losses
    per epoch)."""
    net = SurrogateNet(device, seed=seed)
    model = Surrogate(net, input_stats(train_samples), cheap_divisor=cheap_divisor)
    feats, targets = [], []
    for s in train_samples:
        x, sums = model.features(s[1], s[2], s[3])
        feats.append(x)
        targets.append(model.target(s[3], s[4], sums))
    loss_buf = torch.zeros(1, device=device)
    losses = []
    order = np.arange(len(train_samples))
    rng = np.random.default_rng(seed)
    steps_per_epoch = (len(order) + batch - 1) // batch
    total = epochs * steps_per_epoch
    step = 0
    for ep in range(epochs):
        rng.shuffle(order)
        loss_buf.zero_()
        for b0 in range(0, len(order), batch):
            idx = order[b0:b0 + batch]
            dw = [torch.zeros_like(w) for w in net.w]
            db = [torch.zeros_like(b) for b in net.b]
            for i in idx:
                y, cache = net.forward(feats[i], keep=True)
                dz = torch.empty_like(y)
                rtmi.mse_loss(y, targets[i], 1.0 / (targets[i].numel() * len(idx)), dz, loss_buf)
                net.backward(cache, dz, dw=dw, db=db)
            net.apply(dw, db, learning_rate(lr, step, total, warmup, schedule))
            step += 1
        losses.append(float(loss_buf.item()) / steps_per_epoch)
        if log:
            log(f"epoch {ep}: mean squared log-error {losses[-1]:.3e}")
    return model, losses


def calibrate(model, val_samples, target=0.01):
    """Largest check threshold at which every accepted validation prediction is within
    `target` relative L2 of the full march. Returns (threshold, [(check, true error)])."""
    pairs = []
    for w, j, k, cheap, full in val_samples:
        field, check = model.predict(j, k, cheap)
        pairs.append((check, rel_l2(field, full)))
    pairs.sort()
    thr = 0.0
    for check, err in pairs:
        if err > target:
            break
        thr = check
    model.threshold = thr
    return thr, pairs


def evaluate(model, eval_samples, reps=3):
    """Per-sample outputs of model.run against the full march, and fields/s of the
    surrogate path (with its fallbacks) and of the plain march."""
    errs, used = [], []
    for w, j, k, cheap, full in eval_samples:
        field, u = model.run(w, j, k)
        errs.append(rel_l2(field, full))
        used.append(u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for w, j, k, _, _ in eval_samples:
            model.run(w, j, k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        for w, j, k, _, _ in eval_samples:
            rtmi.trace_multi(j, k, w.source_pos, w.num_rays, w.step_size, w.radiation_velocity, w.time_step)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    # the network's own path (cheap march, features, six convolutions, output), no fallback
    for _ in range(reps):
        for w, j, k, _, _ in eval_samples:
            cheap = rtmi.trace_multi(j, k, w.source_pos, np.maximum(w.num_rays // model.cheap_divisor, 1),
                                     w.step_size, w.radiation_velocity, w.time_step)
            x, sums = model.features(j, k, cheap)
            y, _ = model.net.forward(x)
            rtmi.surrogate_output(y, cheap, sums)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    n = reps * len(eval_samples)
    return {"max_err": max(errs), "mean_err": float(np.mean(errs)), "accepted": int(sum(used)),
            "samples": len(eval_samples), "surrogate_fields_per_s": n / (t1 - t0),
            "march_fields_per_s": n / (t2 - t1), "network_path_fields_per_s": n / (t3 - t2)}


def conv_rates(dev, n=64, reps=20):
    """Milliseconds and TFLOP/s of the four convolution kernels on one n^3 sample with 32
    channels (55,296 flop per voxel and layer), HIP events on the current stream over
    `reps` launches each after warm-up: the forward pass with and without the binary32
    pre-activation kept, the data gradient and the weight gradient (with its transposes).
    Also the bytes each moves at least (bf16 activations, binary32 pre-activations) and
    the resulting HBM rate."""
    g = torch.Generator(device="cpu").manual_seed(0)
    shape = (1, n, n, n, rtmi.CONV_CHANNELS)
    x = (torch.randn(shape, generator=g) * 0.5).to(torch.bfloat16).to(dev)
    w = (torch.randn(rtmi.WEIGHT_SHAPE, generator=g) * 0.05).to(torch.bfloat16).to(dev)
    bias = torch.zeros(rtmi.CONV_CHANNELS, device=dev)
    z = torch.empty(shape, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    dh = torch.empty_like(z)
    dzp = torch.empty_like(x)
    dw = torch.zeros(rtmi.WEIGHT_SHAPE, device=dev)
    db = torch.zeros(rtmi.CONV_CHANNELS, device=dev)
    vox = n ** 3
    flop = 2 * 27 * rtmi.CONV_CHANNELS * rtmi.CONV_CHANNELS * vox
    a16, a32 = 2 * rtmi.CONV_CHANNELS * vox, 4 * rtmi.CONV_CHANNELS * vox   # one activation tensor, bytes

    def timed(fn):
        for _ in range(3):
            fn()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            fn()
        end.record()
        end.synchronize()
        return start.elapsed_time(end) / reps

    kernels = {
        # x and the residual read, y and z written
        "forward": (lambda: rtmi.conv3d_forward(x, w, bias=bias, residual=x, gelu=True, z=z, y=y), 2 * a16 + a16 + a32),
        "forward_no_preactivation": (lambda: rtmi.conv3d_forward(x, w, bias=bias, residual=x, gelu=True, y=y),
                                     3 * a16),
        # dz and the next layer's pre-activation read, dh and dz_prev written
        "backward_data": (lambda: rtmi.conv3d_backward_data(x, w, residual=z, zprev=z, dh=dh, dz_prev=dzp),
                          a16 + a32 + a32 + a16),
        # x and dz read (then their channel-major copies: x three times)
        "backward_weight": (lambda: rtmi.conv3d_backward_weight(x, x, dw, db), 2 * a16),
    }
    out = {}
    for name, (fn, nbytes) in kernels.items():
        ms = timed(fn)
        out[name] = {"ms": ms, "tflops": flop / (ms * 1e-3) / 1e12, "min_bytes": nbytes,
                     "min_bytes_TBps": nbytes / (ms * 1e-3) / 1e12}
    return {"grid": n, "flop_per_layer": flop, "kernels": out}


def main(argv=None):
    """Train, calibrate and evaluate the surrogate on seeded 64^3 turbulent samples (16
    sources, 4096 rays, 128 substeps; training seeds 0.., validation 5000.., evaluation
    10000..) and print a JSON summary."""
    import argparse
    import json
    ap = argparse.ArgumentParser(description=main.__doc__.split("\n")[0])
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--val", type=int, default=100)
    ap.add_argument("--eval", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--target", type=float, default=0.01)
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--schedule", choices=("step", "cosine", "constant"), default="step")
    ap.add_argument("--cheap-divisor", type=int, default=CHEAP_DIVISOR)
    ap.add_argument("--save", default=None, help="checkpoint path for the trained, calibrated surrogate")
    ap.add_argument("--conv-bench", action="store_true", help="only time the convolution kernels at 64^3")
    args = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    if args.conv_bench:
        print(json.dumps(conv_rates(dev)), flush=True)
        return
    t0 = time.perf_counter()
    cd = args.cheap_divisor
    train_s = [make_sample(s, dev, cheap_divisor=cd) for s in range(args.train)]
    val_s = [make_sample(5000 + s, dev, cheap_divisor=cd) for s in range(args.val)]
    eval_s = [make_sample(10000 + s, dev, cheap_divisor=cd) for s in range(args.eval)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"samples ready in {t1 - t0:.1f} s", flush=True)
    model, losses = train(train_s, dev, epochs=args.epochs, lr=args.lr, batch=args.batch, warmup=args.warmup,
                          schedule=args.schedule, cheap_divisor=cd, log=lambda m: print(m, flush=True))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    thr, pairs = calibrate(model, val_s, target=args.target)
    res = evaluate(model, eval_s)
    checks = np.array([p[0] for p in pairs])
    errs = np.array([p[1] for p in pairs])
    cheap = [rel_l2(s[3], s[4]) for s in eval_s]
    if args.save:
        model.save(args.save)
    out = {"train_samples": args.train, "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
           "warmup": args.warmup, "schedule": args.schedule, "cheap_divisor": cd, "train_s": t2 - t1,
           "train_samples_per_s": args.train * args.epochs / (t2 - t1), "losses": losses,
           "threshold": thr, "val_error_median": float(np.median(errs)), "val_error_min": float(errs.min()),
           "val_check_median": float(np.median(checks)), "cheap_error_mean": float(np.mean(cheap)),
           **res}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
