"""Training of the learned block preconditioner (off the sampling path).

The network, its features and the fallback rules are defined with the C ABI
(include/pse.h).  Training regresses the network output y_i onto
T_i - I, where T_i is the normalised symmetric root of the ii block of the
inverse of M_r restricted to particle i's neighbourhood
(pse_precond_targets), with the squared error summed over the 9 entries and
averaged over particles.  Every step of an epoch runs in the HIP library
on the device, with no host synchronisation: the forward pass and the
backward pass on the matrix cores, the loss and its gradient
(pse_mlp_loss_grad) and the Adam step; the loss history is read back once.
"""
import numpy as np

from . import (MLP_NPARAM, _ptr, pse_mlp_adam, pse_mlp_backward, pse_mlp_backward_workspace, pse_mlp_forward,
               pse_mlp_loss_grad, pse_precond_targets)

# (name, rows, cols, stored cols / rows) of the flat weight layout
LAYOUT = (("W1", 64, 24, 32), ("b1", 64, 1, 1), ("W2", 64, 64, 64), ("b2", 64, 1, 1), ("W3", 9, 64, 16),
          ("b3", 9, 1, 16))


def pack(w):
    """Weight dict (W1 (64,24), b1 (64,), W2 (64,64), b2, W3 (9,64), b3 (9,))
    -> flat float32 array of MLP_NPARAM entries with zero padding."""
    out = []
    for name, r, c, stored in LAYOUT:
        a = np.asarray(w[name], dtype=np.float32)
        if name == "W1":
            blk = np.zeros((64, 32), np.float32)
            blk[:, :24] = a
        elif name == "W3":
            blk = np.zeros((16, 64), np.float32)
            blk[:9] = a
        elif name == "b3":
            blk = np.zeros(16, np.float32)
            blk[:9] = a
        else:
            blk = a.reshape(-1)
        out.append(blk.reshape(-1))
    flat = np.concatenate(out)
    assert flat.size == MLP_NPARAM
    return flat


def unpack(flat):
    flat = np.asarray(flat, dtype=np.float64)
    o = 0
    w = {}
    for name, r, c, stored in LAYOUT:
        if name == "W1":
            w[name] = flat[o:o + 64 * 32].reshape(64, 32)[:, :24].copy()
            o += 64 * 32
        elif name == "W3":
            w[name] = flat[o:o + 16 * 64].reshape(16, 64)[:9].copy()
            o += 16 * 64
        elif name == "b3":
            w[name] = flat[o:o + 16][:9].copy()
            o += 16
        else:
            w[name] = flat[o:o + r * c].reshape((r, c) if c > 1 else (r,)).copy()
            o += r * c
    return w


def bf16_bits(a):
    """float32 -> bfloat16 bit patterns (round to nearest even), uint16."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return np.where(np.isnan(np.asarray(a, np.float32)), np.uint16(0x7FC0), r)


def init_weights(seed):
    """He-scaled hidden layers; zero output layer, so that P = I at start."""
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.standard_normal((64, 24)) * np.sqrt(2.0 / 24),
        "b1": np.zeros(64),
        "W2": rng.standard_normal((64, 64)) * np.sqrt(2.0 / 64),
        "b2": np.zeros(64),
        "W3": np.zeros((9, 64)),
        "b3": np.zeros(9),
    }


class Trainer:
    """Accumulates (features, target) rows from sampling contexts created
    with precond=1, then fits the network with Adam on the device."""

    def __init__(self, torch, seed=0, lr=1e-3):
        self.torch = torch
        self.lr = lr
        self.t = 0
        flat = pack(init_weights(seed))
        dev = "cuda"
        self.wm = torch.tensor(flat, dtype=torch.float32, device=dev)
        self.wb = torch.tensor(bf16_bits(flat).view(np.int16), dtype=torch.int16, device=dev).view(torch.bfloat16)
        self.m = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=dev)
        self.v = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=dev)
        self.dw = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=dev)
        self.X = []
        self.T = []

    def add(self, sampler, positions, idx, radius=0.0):
        """Rows for caller indices idx of the sampler's current positions
        (positions: the same (n, 3) array, host)."""
        feat = sampler.precond_features()
        self.X.append(feat[self.torch.as_tensor(np.asarray(idx), device="cuda", dtype=self.torch.long)])
        T = pse_precond_targets(sampler.params, np.asarray(positions, np.float64), idx, radius)
        self.T.append((T - np.eye(3)[None]).reshape(-1, 9))

    def fit(self, epochs, log_every=0):
        torch = self.torch
        X = torch.cat(self.X).contiguous()
        T = torch.as_tensor(np.concatenate(self.T), dtype=torch.float32, device="cuda").contiguous()
        n = len(T)
        losses = torch.zeros(max(epochs, 1), dtype=torch.float32, device="cuda")
        y = torch.empty((n, 9), dtype=torch.float32, device="cuda")
        cache = torch.empty((n, 128), dtype=torch.bfloat16, device="cuda")
        dy = torch.empty((n, 9), dtype=torch.float32, device="cuda")
        wbytes = pse_mlp_backward_workspace(n)
        work = torch.empty(wbytes // 4, dtype=torch.float32, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        P = lambda t, dt, k, nm: _ptr(t, dt, k, nm)
        wb = P(self.wb, torch.bfloat16, MLP_NPARAM, "w")
        xp = P(X, torch.bfloat16, 24 * n, "x")
        yp, cp, dyp = P(y, torch.float32, 9 * n, "y"), P(cache, torch.bfloat16, 128 * n, "cache"), \
            P(dy, torch.float32, 9 * n, "dy")
        tp = P(T, torch.float32, 9 * n, "target")
        for ep in range(epochs):
            pse_mlp_forward(wb, xp, n, yp, cp, stream)
            pse_mlp_loss_grad(yp, tp, n, dyp, P(losses[ep:ep + 1], torch.float32, 1, "loss"), stream)
            pse_mlp_backward(wb, xp, cp, dyp, n, P(self.dw, torch.float32, MLP_NPARAM, "dw"),
                             P(work, torch.float32, wbytes // 4, "work"), wbytes, stream)
            self.t += 1
            pse_mlp_adam(P(self.wm, torch.float32, MLP_NPARAM, "wm"), wb,
                         P(self.dw, torch.float32, MLP_NPARAM, "dw"), P(self.m, torch.float32, MLP_NPARAM, "m"),
                         P(self.v, torch.float32, MLP_NPARAM, "v"), self.lr, self.t, stream)
            if log_every and ep % log_every == 0:
                print(f"[precond] epoch {ep}: loss {float(losses[ep]):.4e}", flush=True)
        torch.cuda.synchronize()
        return [float(v) for v in losses[:epochs].cpu().numpy()]

    def weights_bits(self):
        """The trained bf16 weights as uint16 bit patterns (host)."""
        return self.wb.view(self.torch.int16).cpu().numpy().view(np.uint16)
