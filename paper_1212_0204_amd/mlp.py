"""The closure network (37 -> 64 -> 64 -> 64 -> 4, tanh) and its training.

Argument marshalling over the ``hofks_mlp_*`` and ``hofks_closure_*`` entry
points: parameters, Adam moments, gradient, work areas and the packed BF16
form live in torch device tensors; the target scales, the clipping, the
forward pass, the gradient, Adam, the packing and the scale fold run in the
library's kernels.  Torch allocates and draws the minibatch indices (its
device RNG); it does no arithmetic on the data.
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
        self.work = torch.empty(0, dtype=torch.uint8, device="cuda")
        self.pack()

    def _work(self, nbytes):
        """device scratch of at least nbytes (kept between calls)"""
        if self.work.numel() < nbytes:
            self.work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        return self.work

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
        L = _lib.lib()
        nb = L.hofks_mlp_grad_work_bytes(n)
        w = self._work(nb)
        _check(L.hofks_mlp_grad(_vp(self.packed), _vp(x), _vp(t),
                                _vp(idx) if idx is not None else None, n,
                                _vp(self.grad), _vp(self.loss), _vp(w), nb, self.stream),
               "mlp_grad")
        return self.grad, self.loss

    def train_step(self, x, t, idx, lr, b1=0.9, b2=0.999, eps=1e-8):
        """gradient of the rows idx of (x, t), one Adam step and the packing,
        in one library call; the minibatch loss stays on the device"""
        L = _lib.lib()
        nb = L.hofks_mlp_grad_work_bytes(idx.shape[0])
        w = self._work(nb)
        self.adam_steps += 1
        _check(L.hofks_closure_train_step(_vp(self.params), _vp(self.m), _vp(self.v),
                                          _vp(self.packed), _vp(x), _vp(t), _vp(idx),
                                          idx.shape[0], lr, b1, b2, eps, self.adam_steps,
                                          _vp(self.grad), _vp(self.loss), _vp(w), nb, self.stream),
               "closure_train_step")

    def adam(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.adam_steps += 1
        _check(_lib.lib().hofks_mlp_adam(_vp(self.params), _vp(self.grad), _vp(self.m),
                                         _vp(self.v), lr, b1, b2, eps, self.adam_steps,
                                         self.stream), "mlp_adam")
        self.pack()

    def train(self, x, t, steps, batch=4096, lr=2e-3, lr_end=2e-4, seed=0, log_every=0):
        """minibatch Adam on (x, t) (t already divided by sigma); geometric
        decay of the learning rate from lr to lr_end; returns the logged
        losses"""
        x = x.contiguous()
        t = t.contiguous()
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        losses = []
        for it in range(steps):
            idx = torch.randint(0, x.shape[0], (batch,), device="cuda", generator=g,
                                dtype=torch.int32)
            rate = lr * (lr_end / lr) ** (it / max(steps - 1, 1))
            self.train_step(x, t, idx, rate)
            if log_every and (it % log_every == 0 or it == steps - 1):
                losses.append((it, float(self.loss.item())))
        return losses

    def state(self):
        return self.params.detach().cpu().numpy().copy(), self.sigma

    def prepare(self, x, t, clip=8.0):
        """the training set of the closure snapshots (library call
        hofks_closure_prepare): per-output robust scales, normalised targets,
        samples beyond `clip` left out; returns (x_kept, t_kept, scales)
        with the scales as a (4,) FP64 device tensor"""
        L = _lib.lib()
        x = x.contiguous()
        t = t.contiguous()
        n = x.shape[0]
        xo = torch.empty_like(x)
        to = torch.empty_like(t)
        scales = torch.empty(NOUT, dtype=torch.float64, device="cuda")
        kept = torch.empty(1, dtype=torch.int32, device="cuda")
        nb = L.hofks_closure_prepare_work_bytes(n)
        w = self._work(nb)
        _check(L.hofks_closure_prepare(_vp(x), _vp(t), n, float(clip), _vp(xo), _vp(to),
                                       _vp(scales), _vp(kept), _vp(w), nb, self.stream),
               "closure_prepare")
        k = int(kept.item())
        return xo[:k], to[:k], scales

    def fold_scales(self, scales):
        _check(_lib.lib().hofks_mlp_fold_scales(_vp(self.params), _vp(scales), self.stream),
               "mlp_fold_scales")
        self.pack()

    def fit_closure(self, x, t, steps=4000, batch=4096, lr=2e-3, lr_end=1e-4, clip=8.0, seed=0,
                    log_every=0):
        """Train on closure snapshots with each output normalised by a robust
        scale (the standard deviation of the component after dropping its
        top 0.5% in magnitude); samples with a normalised target beyond
        `clip` are left out (shock cells, which the delta marks keep
        kinetic).  The scales are folded into the output layer afterwards,
        so sigma = 1.  Returns (scales, logged losses, samples used)."""
        xs, ts, scales = self.prepare(x, t, clip)
        self.sigma = 1.0
        losses = self.train(xs, ts, steps, batch=batch, lr=lr, lr_end=lr_end, seed=seed,
                            log_every=log_every)
        self.fold_scales(scales)
        return scales.cpu().numpy().astype(np.float32), losses, int(xs.shape[0])


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
