"""Learned list size: binding of the k-model ABI and its training pipeline.

The network (12 features -> 64 -> 64 -> 7 buckets, BF16 MFMA kernels) is
trained on the GPU by the library's own forward/backward/Adam kernels.  Its
labels are produced by the method itself: each training cell is clipped with
a 64-long list by the label-recording clip kernel, which reports the least
list size at which the security radius certified the cell; the label is the
least bucket {8, 12, 16, 24, 32, 48, 64} that is not smaller (64 when the
cell needs more than 64).  At run time the network's choice only sets how
long each cell's list is: the certificate and the GPU stream phase still
decide the cell, so the tessellation does not depend on the network.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np
import torch

from . import _lib
from ._lib import NPARAM, NFEAT, check

BUCKETS = np.array([8, 12, 16, 24, 32, 48, 64])


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class KModel:
    def __init__(self, ctx=None, seed: int = 0, tau: float = 0.9, _handle=None):
        from . import Context
        self.ctx = ctx or Context.get()
        self.lib = self.ctx.lib
        h = _handle if _handle is not None else self.lib.votess_kmodel_create(self.ctx.handle, seed)
        if not h:
            raise _lib.VotessError(1, self.lib.votess_last_error().decode())
        self.handle = C.c_void_p(h)
        self.tau = tau
        self.history: list[float] = []

    # versioned blob (weights, standardisation, tau) ------------------------
    def save(self) -> bytes:
        n = self.lib.votess_kmodel_blob_size()
        buf = C.create_string_buffer(n)
        ln = C.c_size_t(0)
        check(self.lib.votess_kmodel_save(self.handle, float(self.tau), buf, n, C.byref(ln)))
        return buf.raw[: ln.value]

    @classmethod
    def load(cls, blob: bytes, ctx=None) -> "KModel":
        from . import Context
        ctx = ctx or Context.get()
        h = C.c_void_p()
        tau = C.c_double(0.0)
        check(ctx.lib.votess_kmodel_load(ctx.handle, blob, len(blob), C.byref(h), C.byref(tau)))
        return cls(ctx=ctx, tau=tau.value, _handle=h.value)

    def fit_norm(self, feats: torch.Tensor):
        """Sets the standardisation to the mean / std of ``feats`` [n,12] (on the device)."""
        feats = feats.contiguous()
        check(self.lib.votess_kmodel_fit_norm(self.handle, _ptr(feats), feats.shape[0], _stream()))

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                self.lib.votess_kmodel_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    # parameters -----------------------------------------------------------
    def set_params(self, params=None, mean=None, std=None):
        P = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        M = None if mean is None else np.ascontiguousarray(mean, dtype=np.float32)
        S = None if std is None else np.ascontiguousarray(std, dtype=np.float32)
        if P is not None:
            assert P.shape == (NPARAM,)
        torch.cuda.synchronize()
        check(self.lib.votess_kmodel_set_params(self.handle, None if P is None else P.ctypes.data,
                                                None if M is None else M.ctypes.data,
                                                None if S is None else S.ctypes.data))

    def get_params(self):
        P = np.zeros(NPARAM, np.float32)
        M = np.zeros(NFEAT, np.float32)
        S = np.zeros(NFEAT, np.float32)
        torch.cuda.synchronize()
        check(self.lib.votess_kmodel_get_params(self.handle, P.ctypes.data, M.ctypes.data, S.ctypes.data))
        return P, M, S

    # kernels ---------------------------------------------------------------
    def forward(self, feats: torch.Tensor) -> torch.Tensor:
        feats = feats.contiguous()
        out = torch.empty(max(feats.shape[0], 1), 7, dtype=torch.float32, device=feats.device)
        check(self.lib.votess_kmodel_forward(self.handle, _ptr(feats), feats.shape[0], _ptr(out), _stream()))
        return out[: feats.shape[0]]

    def choose(self, feats: torch.Tensor, tau: float | None = None) -> torch.Tensor:
        feats = feats.contiguous()
        out = torch.empty(max(feats.shape[0], 1), dtype=torch.uint8, device=feats.device)
        check(self.lib.votess_kmodel_choose(self.handle, _ptr(feats), feats.shape[0],
                                            float(self.tau if tau is None else tau), _ptr(out), _stream()))
        return out[: feats.shape[0]]

    def grad(self, feats: torch.Tensor, labels: torch.Tensor):
        g = torch.empty(NPARAM, dtype=torch.float32, device=feats.device)
        loss = torch.empty(1, dtype=torch.float32, device=feats.device)
        check(self.lib.votess_kmodel_grad(self.handle, _ptr(feats.contiguous()), _ptr(labels.contiguous()),
                                          feats.shape[0], _ptr(g), _ptr(loss), _stream()))
        return g, loss

    def train_step(self, feats: torch.Tensor, labels: torch.Tensor, lr: float = 1e-3) -> torch.Tensor:
        loss = torch.empty(1, dtype=torch.float32, device=feats.device)
        check(self.lib.votess_kmodel_train_step(self.handle, _ptr(feats), _ptr(labels), feats.shape[0],
                                                float(lr), _ptr(loss), _stream()))
        return loss


def features(sorted_, grid, cell_start, queries=None, ctx=None) -> torch.Tensor:
    """12 features per query (F32 sorted points)."""
    from . import Context, _grid_c, _sub
    ctx = ctx or Context.get()
    n = sorted_.shape[0]
    nq = n if queries is None else queries.shape[0]
    out = torch.empty(max(nq, 1), NFEAT, dtype=torch.float32, device=sorted_.device)
    si, ss = _sub(grid)
    check(ctx.lib.votess_features(ctx.handle, _ptr(sorted_), n, C.byref(_grid_c(grid)), _ptr(cell_start), si, ss,
                                  _ptr(queries), nq, _ptr(out), _stream()))
    return out[:nq]


def labels(status: torch.Tensor, kneeded: torch.Tensor, ctx=None) -> torch.Tensor:
    """Bucket label per cell from the label-recording clip (library kernel)."""
    from . import Context
    ctx = ctx or Context.get()
    n = status.shape[0]
    out = torch.empty(max(n, 1), dtype=torch.uint8, device=status.device)
    check(ctx.lib.votess_kmodel_labels(ctx.handle, _ptr(status.contiguous()), _ptr(kneeded.contiguous()), n,
                                       _ptr(out), _stream()))
    return out[:n]


def method_labels(sorted_, grid, cell_start, cells, precision: str = "f32"):
    """Bucket labels from the method: least bucket >= the certifying list size
    (the largest bucket when a 64-long list does not certify the cell)."""
    from . import clip_cells, knn
    lists = knn(sorted_, grid, cell_start, 64, queries=cells, dist="f32" if precision != "f64" else "f64")
    r = clip_cells(sorted_, lists, 64, cells=cells, precision=precision, kneeded=True)
    st, kn = r["status"], r["kneeded"]
    cap = torch.nonzero(st == 2).flatten()
    if cap.numel():  # overflow of the fast kernel: same lists, large-capacity kernel
        rc = clip_cells(sorted_, lists[cap].contiguous(), 64, cells=cells[cap].contiguous(), precision=precision,
                        kneeded=True, capacity=1)
        st = st.clone()
        kn = kn.clone()
        st[cap] = rc["status"]
        kn[cap] = rc["kneeded"]
    return labels(st, kn), kn


def train(points: torch.Tensor, box=((0, 0, 0), (1, 1, 1)), n_train: int = 1 << 21, epochs: int = 4,
          batch: int = 8192, lr: float = 1e-3, seed: int = 1, precision: str = "f32", log=None) -> KModel:
    """Trains a k-model on the method's own labels for n_train cells of ``points``."""
    from . import grid_sort
    t0 = time.time()
    cs, perm, srt, grid = grid_sort(points, box)
    n = points.shape[0]
    rng = np.random.default_rng(seed)
    cells_np = np.sort(rng.choice(n, size=min(n_train, n), replace=False)).astype(np.int32)
    cells = torch.from_numpy(cells_np).to(points.device)
    X = features(srt, grid, cs, cells)
    lab, kn = method_labels(srt, grid, cs, cells, precision)
    model = KModel(seed=seed)
    model.fit_norm(X)
    order = torch.from_numpy(rng.permutation(len(cells_np))).to(points.device)
    Xs = X[order].contiguous()
    Ys = lab[order].contiguous()
    nb = len(cells_np) // batch
    t1 = time.time()
    for ep in range(epochs):
        losses = []
        for b in range(nb):
            losses.append(model.train_step(Xs[b * batch:(b + 1) * batch], Ys[b * batch:(b + 1) * batch], lr))
        ep_loss = float(torch.stack(losses).mean().item())
        model.history.append(ep_loss)
        if log:
            log(f"[kmodel] epoch {ep + 1}/{epochs} loss {ep_loss:.4f}")
    torch.cuda.synchronize()
    model.train_seconds = time.time() - t1
    model.prep_seconds = t1 - t0
    model.label_hist = torch.bincount(lab.long(), minlength=7).cpu().tolist()
    return model


def tune_tau(model: KModel, points: torch.Tensor, taus=(0.5, 0.7, 0.8, 0.9, 0.95), precision="f32", log=None,
             max_gpu_retries: int = 0):
    """Picks the threshold with the fastest learned tessellation of ``points``
    (a validation set, not the evaluation input), with the given number of
    k doublings after the learned pass."""
    from . import tessellate
    best = None
    kw = dict(precision=precision, kmodel=model, max_gpu_retries=max_gpu_retries)
    for tau in taus:
        tessellate(points, tau=tau, **kw)  # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        tessellate(points, tau=tau, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        if log:
            log(f"[kmodel] tau {tau}: {dt * 1e3:.1f} ms")
        if best is None or dt < best[1]:
            best = (tau, dt)
    model.tau = best[0]
    return best


_cache: dict = {}


def load_default(workload: str, log=None, max_gpu_retries: int = 0) -> KModel:
    """A model for a named workload: trained on 2^21 cells of the workload's
    seed-1 point set, tau tuned on that set (the evaluation input is seed 0)
    for runs with ``max_gpu_retries`` doublings of k after the learned pass."""
    key = (workload, max_gpu_retries)
    if key in _cache:
        return _cache[key]
    from . import gen
    P = torch.from_numpy(gen.make(workload, seed=1)).cuda()
    model = train(P, log=log)
    tune_tau(model, P, log=log, max_gpu_retries=max_gpu_retries)
    del P
    _cache[key] = model
    return model
