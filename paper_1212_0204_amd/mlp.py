"""The closure network (37 -> 64 -> 64 -> 64 -> 4, tanh) and its training.

Argument marshalling over the ``hofks_mlp_*`` entry points: parameters,
Adam moments, gradient and the packed BF16 form live in torch device tensors;
forward, gradient, Adam and packing run in the library's kernels.  Torch
draws the minibatch indices (its device RNG) and nothing else.
"""
import ctypes

import numpy as np
import torch

from . import _lib

NIN, NH, NOUT = 37, 64, 4
SHAPES = [(NH, NIN), (NH,), (NH, NH), (NH,), (NH, NH), (NH,), (NOUT, NH), (NOUT,)]


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def _check(st, what):
    if st != 0:
        from .solver import HofksError
        raise HofksError(st, what)


def init_params(seed=0):
    """Glorot-uniform weights, zero biases, in the flat FP32 layout"""
    rng = np.random.default_rng(seed)
    out = []
    for shp in SHAPES:
        if len(shp) == 2:
            a = np.sqrt(6.0 / (shp[0] + shp[1]))
            out.append(rng.uniform(-a, a, shp).ravel())
        else:
            out.append(np.zeros(shp))
    return np.concatenate(out).astype(np.float32)


class ClosureNet:
    """FP32 master parameters + Adam state on the GPU, packed BF16 weights
    for the kernels, and the output scale ``sigma`` (the network predicts
    targets / sigma)."""

    def __init__(self, params=None, sigma=1.0, seed=0):
        L = _lib.lib()
        self.nparam = L.hofks_mlp_nparam()
        p = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        assert p.shape == (self.nparam,)
        self.params = torch.tensor(p, device="cuda")
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.packed = torch.empty(L.hofks_mlp_packed_bytes(), dtype=torch.uint8, device="cuda")
        self.sigma = float(sigma)
        self.adam_steps = 0
        self.pack()

    @property
    def stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def pack(self):
        _check(_lib.lib().hofks_mlp_pack(_vp(self.params), _vp(self.packed), self.stream), "mlp_pack")

    def forward(self, x):
        """network output for x (n x 37 FP32 device tensor)"""
        x = x.contiguous()
        y = torch.empty((x.shape[0], NOUT), dtype=torch.float32, device="cuda")
        _check(_lib.lib().hofks_mlp_forward(_vp(self.packed), _vp(x), _vp(y), x.shape[0],
                                            self.stream), "mlp_forward")
        return y

    def gradient(self, x, t, idx=None):
        """(grad, loss) of the mean squared error over the rows idx of x, t
        (all rows without idx); device tensors, valid until the next call"""
        n = x.shape[0] if idx is None else idx.shape[0]
        _check(_lib.lib().hofks_mlp_grad(_vp(self.packed), _vp(x), _vp(t),
                                         _vp(idx) if idx is not None else None, n,
                                         _vp(self.grad), _vp(self.loss), self.stream), "mlp_grad")
        return self.grad, self.loss

    def adam(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.adam_steps += 1
        _check(_lib.lib().hofks_mlp_adam(_vp(self.params), _vp(self.grad), _vp(self.m),
                                         _vp(self.v), lr, b1, b2, eps, self.adam_steps,
                                         self.stream), "mlp_adam")
        self.pack()

    def train(self, x, t, steps, batch=4096, lr=2e-3, lr_end=2e-4, seed=0, log_every=0):
        """minibatch Adam on (x, t / sigma); cosine-free geometric decay of the
        learning rate from lr to lr_end; returns the logged losses"""
        x = x.contiguous()
        ts = (t / self.sigma).contiguous()
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        losses = []
        for it in range(steps):
            idx = torch.randint(0, x.shape[0], (batch,), device="cuda", generator=g,
                                dtype=torch.int32)
            self.gradient(x, ts, idx)
            rate = lr * (lr_end / lr) ** (it / max(steps - 1, 1))
            self.adam(rate)
            if log_every and (it % log_every == 0 or it == steps - 1):
                losses.append((it, float(self.loss.item())))
        return losses

    def state(self):
        return self.params.detach().cpu().numpy().copy(), self.sigma

    def fit_closure(self, x, t, steps=4000, batch=4096, lr=2e-3, lr_end=1e-4, clip=8.0, seed=0,
                    log_every=0):
        """Train on closure snapshots with each output normalised by a robust
        scale (the standard deviation of the component after dropping its
        top 0.5% in magnitude); samples with a normalised target beyond
        `clip` are left out (shock cells, which the delta marks keep
        kinetic).  The scales are folded into the output layer afterwards,
        so sigma = 1.  Returns (scales, logged losses, samples used)."""
        ta = t.abs()
        q = torch.quantile(ta[torch.randperm(t.shape[0], device=t.device)[:200000]], 0.995, dim=0)
        sc = torch.stack([t[:, c][ta[:, c] <= q[c]].std() for c in range(NOUT)])
        sc = torch.clamp(sc, min=1e-12)
        tn = t / sc
        keep = (tn.abs() <= clip).all(dim=1)
        xs, ts = x[keep].contiguous(), tn[keep].contiguous()
        self.sigma = 1.0
        losses = self.train(xs, ts, steps, batch=batch, lr=lr, lr_end=lr_end, seed=seed,
                            log_every=log_every)
        p = self.params.detach().cpu().numpy().copy()
        scale = sc.cpu().numpy().astype(np.float32)
        o_w4 = NH * NIN + NH + 2 * (NH * NH + NH)
        p[o_w4:o_w4 + NOUT * NH] *= np.repeat(scale, NH)
        p[o_w4 + NOUT * NH:] *= scale
        self.params.copy_(torch.tensor(p, device="cuda"))
        self.pack()
        return scale, losses, int(keep.sum())


def collect_snapshots(configs, steps_at, precision=1):
    """Training pairs from plain runs: for each configuration (a
    ``workloads.ClosureRun``) the network inputs of U^n and the targets
    N / (lambda s) at the steps listed in ``steps_at`` (device tensors)."""
    from .solver import Solver
    xs, ts = [], []
    for cfg in configs:
        s = Solver(2, (cfg.n, cfg.n), cfg.length / cfg.n, cfg.nv, cfg.dv, bc=(0, 0),
                   precision=precision, tau=cfg.tau)
        s.set_state_macro(*cfg.fields())
        done = 0
        for k in sorted(steps_at):
            if k > done:
                s.step(k - done)
                done = k
            x, t = s.closure_snapshot()
            done += 1
            xs.append(x)
            ts.append(t)
        s.sync()
        del s
    return torch.cat(xs), torch.cat(ts)
