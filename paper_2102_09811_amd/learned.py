"""Learned sparse-approximate-inverse preconditioner for V_h w = b.

A 3-layer tanh MLP (width 256, float32) maps the local data of a row l (near-field entries of
V_h^0 on the row's touching-panel pattern and the local geometry, see ``hb_precond_features``) to
the scaled weights y = V^0[l,l] M[l, pattern] of a sparse approximate inverse M ~ (V_h^0)^{-1}.
Training minimises the mean row residual ||(M V^0)_l - e_l||^2 = y^T G_l y - 2 a_l^T y + 1,
whose G_l, a_l come from ``hb_precond_spai`` on method-generated V^0 blocks (random ellipsoids).
Inference needs only local data; M is then installed with ``hb_precond_set`` and used as the
block-diagonal right preconditioner of GMRES.

Training (shuffling, batching, forward, backward, loss, Adam and the epoch loop) runs in the
library (hb_precond_train); the network is a library object (hb_pcnet) that can be saved, loaded
and installed on a context (hb_precond_install).  The MLP class below drives the single forward /
backward / Adam kernels one call at a time, for checks against the oracle.
"""
import ctypes

import numpy as np

from . import binding as B

N_IN, N_HIDDEN, N_OUT = B.HB_PC_FEATURES, 256, B.HB_PC_SLOTS


def _dims(n_in=N_IN, n_hidden=N_HIDDEN, n_out=N_OUT):
    d = B.MLPDims()
    d.n_in, d.n_hidden, d.n_out = n_in, n_hidden, n_out
    return d


class MLP:
    """Parameters on the device: W1 [H][I], b1 [H], W2 [H][H], b2 [H], W3 [O][H], b3 [O]."""

    def __init__(self, n_in=N_IN, n_hidden=N_HIDDEN, n_out=N_OUT, seed=0, params=None):
        import torch
        self.dims = _dims(n_in, n_hidden, n_out)
        n = B.lib().hb_mlp_num_params(ctypes.byref(self.dims))
        if params is None:
            rng = np.random.default_rng(seed)
            parts = []
            for fan_in, fan_out in ((n_in, n_hidden), (n_hidden, n_hidden), (n_hidden, n_out)):
                lim = np.sqrt(6.0 / (fan_in + fan_out))
                parts.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
                parts.append(np.zeros(fan_out))
            params = np.concatenate(parts).astype(np.float32)
        params = np.ascontiguousarray(params, dtype=np.float32)
        assert params.size == n, (params.size, n)
        self.params = torch.from_numpy(params).cuda()
        self.n = n

    def work(self, batch):
        import torch
        nw = B.lib().hb_mlp_work_floats(ctypes.byref(self.dims), batch)
        return torch.empty(nw, dtype=torch.float32, device="cuda")

    def forward(self, x, work=None, stream=None):
        import torch
        batch = x.shape[0]
        work = self.work(batch) if work is None else work
        y = torch.empty((batch, self.dims.n_out), dtype=torch.float32, device="cuda")
        rc = B.lib().hb_mlp_forward(ctypes.byref(self.dims), B._ptr(self.params), B._ptr(x), batch,
                                    B._ptr(y), B._ptr(work), B._stream(stream))
        if rc != 0:
            raise B.HBError(rc, "hb_mlp_forward")
        return y, work

    def backward(self, x, work, dy, grads=None, stream=None):
        import torch
        grads = torch.empty_like(self.params) if grads is None else grads
        rc = B.lib().hb_mlp_backward(ctypes.byref(self.dims), B._ptr(self.params), B._ptr(x),
                                     x.shape[0], B._ptr(work), B._ptr(dy), B._ptr(grads),
                                     B._stream(stream))
        if rc != 0:
            raise B.HBError(rc, "hb_mlp_backward")
        return grads

    def save(self, path):
        np.savez(path, params=self.params.cpu().numpy(),
                 dims=np.array([self.dims.n_in, self.dims.n_hidden, self.dims.n_out]))

    @classmethod
    def load(cls, path):
        z = np.load(path)
        d = z["dims"]
        return cls(int(d[0]), int(d[1]), int(d[2]), params=z["params"])


def quad_loss(y, G, a, want_grad=True, stream=None):
    """Per-row loss y^T G y - 2 a^T y + 1 and the gradient of its mean w.r.t. y."""
    import torch
    rows = y.shape[0]
    dy = torch.empty_like(y) if want_grad else None
    rl = torch.empty(rows, dtype=torch.float32, device="cuda")
    rc = B.lib().hb_precond_loss(B._ptr(y), B._ptr(G), B._ptr(a), rows,
                                 B._ptr(dy) if want_grad else None, B._ptr(rl), B._stream(stream))
    if rc != 0:
        raise B.HBError(rc, "hb_precond_loss")
    return rl, dy


class Adam:
    def __init__(self, mlp, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        import torch
        self.mlp, self.lr, self.b1, self.b2, self.eps = mlp, lr, beta1, beta2, eps
        self.m = torch.zeros_like(mlp.params)
        self.v = torch.zeros_like(mlp.params)
        self.t = 0

    def step(self, grads, stream=None):
        self.t += 1
        rc = B.lib().hb_adam_step(B._ptr(self.mlp.params), B._ptr(grads), B._ptr(self.m),
                                  B._ptr(self.v), self.mlp.n, self.lr, self.b1, self.b2, self.eps,
                                  self.t, B._stream(stream))
        if rc != 0:
            raise B.HBError(rc, "hb_adam_step")


def mesh_data(verts, tris, alpha, h):
    """Features, Gram matrices, right-hand sides and exact weights of one mesh's V^0 (a one-step
    context with T = h has the same V^0 as any E_t-step problem with that h)."""
    ctx = B.Context(verts, tris, alpha, h, 1)
    ctx.assemble(B.HB_OP_V)
    X = ctx.precond_features()
    G, a, y = ctx.precond_spai(exact=True)
    ctx.close()
    return X, G, a, y


def ellipsoid_set(seeds, n_t=64, T=1.0):
    """The random ellipsoids of the learned-preconditioner workload: semi-axes U[0.5, 2]^3,
    cubed-sphere resolution n in 13..20 (12 n^2 triangles), alpha log-uniform in [0.1, 10]."""
    from synthetic import cubed_sphere_ellipsoid
    out = []
    for sd in seeds:
        rng = np.random.default_rng(1000 + sd)
        axes = rng.uniform(0.5, 2.0, size=3)
        n = int(rng.integers(13, 21))
        alpha = float(10.0 ** rng.uniform(-1.0, 1.0))
        v, t = cubed_sphere_ellipsoid(n, axes)
        out.append({"seed": sd, "verts": v, "tris": t, "alpha": alpha, "h": T / n_t, "n": n,
                    "axes": axes})
    return out


def train(meshes, epochs=30, batch=2048, lr=1e-3, seed=0, log=None):
    """Train the network on the rows of all meshes (hb_precond_train on one-step contexts, which
    carry the same V^0 as any E_t-step problem with that h); returns (PCNet, per-epoch mean
    losses)."""
    ctxs = []
    for m in meshes:
        ctx = B.Context(m["verts"], m["tris"], m["alpha"], m["h"], 1)
        ctx.assemble(B.HB_OP_V)
        ctxs.append(ctx)
    net, hist = B.precond_train(ctxs, epochs=epochs, batch=batch, lr=lr, seed=seed)
    for ctx in ctxs:
        ctx.close()
    if log:
        for ep, L in enumerate(hist):
            log("epoch %d: mean row loss %.4e" % (ep, L))
    return net, hist


def predict(mlp, ctx):
    """Scaled weights [E_x][HB_PC_SLOTS] for the context's assembled V^0 (local data only), with
    the per-call MLP kernels."""
    X = ctx.precond_features()
    y, _ = mlp.forward(X)
    return y


def install(net, ctx):
    """Install the learned preconditioner on ctx: a PCNet through hb_precond_install, an MLP
    through its forward pass and hb_precond_set."""
    if isinstance(net, B.PCNet):
        ctx.precond_install(net)
    else:
        ctx.precond_set(predict(net, ctx))


def evaluate(mlp, meshes, n_t=64, T=1.0, tol=1e-8, log=None):
    """GMRES on the Dirichlet system of each mesh (data exp(alpha t + x.e), E_t steps): plain,
    with the learned preconditioner, and with the exact sparse approximate inverse on the same
    pattern.  Returns one record per mesh (iterations and solve seconds)."""
    import torch
    from synthetic import exp_solution, nodal_samples
    out = []
    for m in meshes:
        v, t, alpha = m["verts"], m["tris"], m["alpha"]
        ctx = B.Context(v, t, alpha, T, n_t)
        ctx.assemble()
        g = nodal_samples(v, n_t, T, lambda x, tt: exp_solution(x, tt, alpha))
        b = ctx.rhs_dirichlet(torch.from_numpy(g).cuda())
        _, ip = ctx.solve(b, method=B.HB_SOLVE_GMRES, tol=tol)
        install(mlp, ctx)
        _, il = ctx.solve(b, method=B.HB_SOLVE_GMRES, tol=tol, precond=True)
        _, _, yex = ctx.precond_spai(exact=True)
        ctx.precond_set(yex)
        _, ie = ctx.solve(b, method=B.HB_SOLVE_GMRES, tol=tol, precond=True)
        rec = {"seed": m["seed"], "E_x": len(t), "alpha": alpha,
               "plain_it": ip["iterations"], "plain_s": ip["seconds"],
               "learned_it": il["iterations"], "learned_s": il["seconds"],
               "learned_res": il["rel_residual"], "exact_spai_it": ie["iterations"]}
        out.append(rec)
        if log:
            log("seed %(seed)d E_x=%(E_x)d alpha=%(alpha).3f: plain %(plain_it)d it, learned "
                "%(learned_it)d it, exact SPAI %(exact_spai_it)d it" % rec)
        ctx.close()
        torch.cuda.empty_cache()
    return out


def main(argv=None):
    """Train on ellipsoid seeds 0 .. n_train-1, evaluate on seeds 160 .. 160+n_test-1."""
    import argparse
    import json
    import sys
    import time
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--train", type=int, default=160)
    ap.add_argument("--test", type=int, default=40)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--save", default=None, help="write the trained network (hb_pcnet_save)")
    args = ap.parse_args(argv)

    def log(msg):
        print("[learned] " + msg, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    train_set = ellipsoid_set(range(args.train))
    log("training on %d ellipsoids (%d rows)" % (len(train_set), sum(len(m["tris"]) for m in train_set)))
    mlp, hist = train(train_set, epochs=args.epochs)
    t_train = time.perf_counter() - t0
    log("trained in %.1f s, loss %.3e -> %.3e" % (t_train, hist[0], hist[-1]))
    if args.save:
        mlp.save(args.save)  # the network file of hb_pcnet_save
    recs = evaluate(mlp, ellipsoid_set(range(160, 160 + args.test)), log=log)
    mean = lambda k: float(np.mean([r[k] for r in recs]))
    summary = {"train_meshes": args.train, "test_meshes": args.test, "epochs": args.epochs,
               "train_seconds": t_train, "loss_first": hist[0], "loss_last": hist[-1],
               "mean_plain_it": mean("plain_it"), "mean_learned_it": mean("learned_it"),
               "mean_exact_spai_it": mean("exact_spai_it"), "mean_plain_s": mean("plain_s"),
               "mean_learned_s": mean("learned_s"), "meshes": recs}
    print(json.dumps(summary), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
