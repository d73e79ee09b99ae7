"""CNN oracle — TEST INFRASTRUCTURE ONLY (imported by the tests and nothing else).

Plain NumPy U-Net: 3x3 cross-correlation with zero padding, bias and ReLU,
2x2 max pooling (ties go to the first element in row-major order), 2x2
stride-2 transposed convolution + ReLU, channel concatenation
[encoder | upsampled], 1x1 linear head, residual output x + f(x), mean
squared error, hand-derived backward pass and Adam.  Each conv is written as
nine shifted matrix products (one per kernel tap); there is no blocking or
fusion.

mode "fp64": everything in double precision.
mode "bf16": emulates a BF16-storage / FP32-accumulate network: the input,
every conv / transposed-conv weight, every stored activation and every stored
activation gradient is rounded to BF16 (round to nearest even) at the point
where it is stored; sums are exact (FP64).

acc "fp32" (either mode) instead forms every convolution, transposed
convolution and their gradients as FP32 matrix products with FP32 results
(the accumulation order is the BLAS library's); "fp32rev" does the same with
the kernel taps (and transposed-conv phases) summed in reverse order.  The
spread between these accumulations and the exact one measures how far two
correct FP32-accumulating implementations may drift apart, which sets the
whole-network tolerance of the GPU tests.

Parameter layout (flat vector): per level l = 0..L-1 the encoder convs a and b,
then per level l = L-2..0 the transposed conv and decoder convs a and b, then
the head.  Conv weights [c_out][3 ty + tx][c_in] then bias; transposed conv
[2 dy + dx][c_out][c_in] then bias; head [c_0] then one bias.  The first conv
reads an 8-channel input whose channel 0 is the image.
"""
from __future__ import annotations

import numpy as np


def to_bf16(a):
    """Round to the nearest BF16 value (ties to even), via FP32; returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def layers(base: int, levels: int):
    out, off = [], 0

    def add(name, kind, cin, cout):
        nonlocal off
        nw = 9 * cin * cout if kind == "conv" else (4 * cin * cout if kind == "up" else cin)
        nb = cout if kind != "head" else 1
        out.append(dict(name=name, kind=kind, cin=cin, cout=cout, w=off, b=off + nw))
        off += nw + nb

    for l in range(levels):
        add(f"enc{l}a", "conv", 8 if l == 0 else base * 2 ** (l - 1), base * 2 ** l)
        add(f"enc{l}b", "conv", base * 2 ** l, base * 2 ** l)
    for l in range(levels - 2, -1, -1):
        c = base * 2 ** l
        add(f"up{l}", "up", 2 * c, c)
        add(f"dec{l}a", "conv", 2 * c, c)
        add(f"dec{l}b", "conv", c, c)
    add("head", "head", base, 1)
    return {d["name"]: d for d in out}, off


class UNetOracle:
    def __init__(self, base: int, levels: int, mode: str = "fp64", acc: str = "fp64"):
        assert mode in ("fp64", "bf16") and acc in ("fp64", "fp32", "fp32rev")
        self.base, self.L, self.mode = base, levels, mode
        self.dt = np.float64 if acc == "fp64" else np.float32
        self.taps = list(range(9))[::-1] if acc == "fp32rev" else list(range(9))
        self.lay, self.n_params = layers(base, levels)

    # rounding at storage points
    def st(self, a):
        return to_bf16(a) if self.mode == "bf16" else a

    def weights(self, p, name):
        d = self.lay[name]
        W = p[d["w"]:d["b"]].astype(np.float64)
        b = p[d["b"]:d["b"] + (d["cout"] if d["kind"] != "head" else 1)].astype(np.float64)
        if d["kind"] == "conv":
            W = W.reshape(d["cout"], 9, d["cin"])
        elif d["kind"] == "up":
            W = W.reshape(4, d["cout"], d["cin"])
        if d["kind"] != "head" and self.mode == "bf16":
            W = to_bf16(W)
        return W, b

    # ---------------------------------------------------------------- layers
    # (operands and sums in self.dt: FP64, or FP32 for the accumulation-spread measurement; results
    # are returned as float64)
    def conv(self, x, W, b):
        """x [B,H,W,Ci], W [Co,9,Ci] -> pre-activation [B,H,W,Co]."""
        dt = self.dt
        B, H, Wd, _ = x.shape
        xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0))).astype(dt)
        W = W.astype(dt)
        out = np.zeros((B, H, Wd, W.shape[0]), dtype=dt) + b.astype(dt)
        for t in self.taps:
            ty, tx = divmod(t, 3)
            out += xp[:, ty:ty + H, tx:tx + Wd, :] @ W[:, t, :].T
        return out.astype(np.float64)

    def conv_bwd(self, x, W, dz):
        """dz at the conv output (already through the ReLU mask) -> (dW, db, dX before masking)."""
        dt = self.dt
        B, H, Wd, Ci = x.shape
        xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0))).astype(dt)
        W, dz = W.astype(dt), dz.astype(dt)
        dW = np.zeros_like(W)
        dxp = np.zeros_like(xp)
        dz2 = dz.reshape(-1, dz.shape[-1])
        for t in self.taps:
            ty, tx = divmod(t, 3)
            dW[:, t, :] = dz2.T @ xp[:, ty:ty + H, tx:tx + Wd, :].reshape(-1, Ci)
            dxp[:, ty:ty + H, tx:tx + Wd, :] += dz @ W[:, t, :]
        f = np.float64
        return dW.astype(f), dz2.sum(axis=0).astype(f), dxp[:, 1:-1, 1:-1, :].astype(f)

    def up(self, x, U, b):
        dt = self.dt
        B, h, w, _ = x.shape
        x, U, b = x.astype(dt), U.astype(dt), b.astype(dt)
        out = np.zeros((B, 2 * h, 2 * w, U.shape[1]), dtype=dt)
        for dy in range(2):
            for dx in range(2):
                out[:, dy::2, dx::2, :] = x @ U[2 * dy + dx].T + b
        return out.astype(np.float64)

    def up_bwd(self, x, U, dy_):
        dt = self.dt
        Ci = x.shape[-1]
        x, U, dy_ = x.astype(dt), U.astype(dt), dy_.astype(dt)
        dU = np.zeros_like(U)
        dx = np.zeros_like(x)
        for ph in (range(4) if self.taps[0] == 0 else range(3, -1, -1)):
            dy, dxx = divmod(ph, 2)
            g = dy_[:, dy::2, dxx::2, :]
            dU[ph] = g.reshape(-1, g.shape[-1]).T @ x.reshape(-1, Ci)
            dx += g @ U[ph]
        f = np.float64
        return dU.astype(f), dy_.reshape(-1, dy_.shape[-1]).sum(axis=0).astype(f), dx.astype(f)

    @staticmethod
    def pool(x):
        B, H, W, C = x.shape
        win = x.reshape(B, H // 2, 2, W // 2, 2, C).transpose(0, 1, 3, 2, 4, 5).reshape(B, H // 2, W // 2, 4, C)
        return win.max(axis=3), win.argmax(axis=3)      # argmax: first maximum in (0,0),(0,1),(1,0),(1,1)

    @staticmethod
    def unpool_add(de, dp, arg, mx):
        """add dp at the argmax of each window into de (only where the maximum is positive)."""
        B, H, W, C = de.shape
        g = np.where(mx > 0, dp, 0.0)
        win = np.zeros((B, H // 2, W // 2, 4, C))
        np.put_along_axis(win, arg[:, :, :, None, :], g[:, :, :, None, :], axis=3)
        return win.reshape(B, H // 2, W // 2, 2, 2, C).transpose(0, 1, 3, 2, 4, 5).reshape(B, H, W, C)

    # ---------------------------------------------------------------- network
    def forward(self, p, x, keep=False):
        """x [B,H,W] -> x + f(x) [B,H,W]."""
        L, st = self.L, self.st
        B, H, W = x.shape
        x8 = np.zeros((B, H, W, 8))
        x8[..., 0] = st(x)
        acts = {"x8": x8}
        cur = x8
        for l in range(L):
            Wa, ba = self.weights(p, f"enc{l}a")
            a = st(np.maximum(self.conv(cur, Wa, ba), 0.0))
            Wb, bb = self.weights(p, f"enc{l}b")
            e = st(np.maximum(self.conv(a, Wb, bb), 0.0))
            acts[f"ea{l}"], acts[f"e{l}"] = a, e
            if l < L - 1:
                cur, arg = self.pool(e)
                acts[f"p{l}"], acts[f"arg{l}"] = cur, arg
        below = acts[f"e{L - 1}"]
        for l in range(L - 2, -1, -1):
            U, bu = self.weights(p, f"up{l}")
            u = st(np.maximum(self.up(below, U, bu), 0.0))
            cat = np.concatenate([acts[f"e{l}"], u], axis=-1)
            Wa, ba = self.weights(p, f"dec{l}a")
            da = st(np.maximum(self.conv(cat, Wa, ba), 0.0))
            Wb, bb = self.weights(p, f"dec{l}b")
            db = st(np.maximum(self.conv(da, Wb, bb), 0.0))
            acts[f"cat{l}"], acts[f"da{l}"], acts[f"db{l}"] = cat, da, db
            below = db
        wh, bh = self.weights(p, "head")
        out = x.astype(np.float64) + (bh[0] + below @ wh)
        return (out, acts) if keep else out

    def loss_and_grad(self, p, x, t):
        """MSE loss and the flat gradient with respect to p."""
        L, st = self.L, self.st
        out, A = self.forward(p, x, keep=True)
        n = out.size
        loss = float(np.mean((out - t) ** 2))
        dout = 2.0 * (out - t) / n
        g = np.zeros(self.n_params)

        def put(name, dW, db):
            d = self.lay[name]
            g[d["w"]:d["b"]] = dW.ravel()
            g[d["b"]:d["b"] + db.size] = db

        wh, _ = self.weights(p, "head")
        d0 = A["db0"]
        put("head", (d0 * dout[..., None]).reshape(-1, d0.shape[-1]).sum(0), np.array([dout.sum()]))
        d_db = st(np.where(d0 > 0, dout[..., None] * wh, 0.0))
        d_skip = {}
        for l in range(0, L - 1):
            Wb, _ = self.weights(p, f"dec{l}b")
            dW, db_, dx = self.conv_bwd(A[f"da{l}"], Wb, d_db)
            put(f"dec{l}b", dW, db_)
            d_da = st(np.where(A[f"da{l}"] > 0, dx, 0.0))
            Wa, _ = self.weights(p, f"dec{l}a")
            dW, db_, dx = self.conv_bwd(A[f"cat{l}"], Wa, d_da)
            put(f"dec{l}a", dW, db_)
            d_cat = st(np.where(A[f"cat{l}"] > 0, dx, 0.0))
            c = self.base * 2 ** l
            d_skip[l] = d_cat[..., :c]
            below = A[f"db{l + 1}"] if l + 1 < L - 1 else A[f"e{L - 1}"]
            U, _ = self.weights(p, f"up{l}")
            dU, dbu, dx = self.up_bwd(below, U, d_cat[..., c:])
            put(f"up{l}", dU, dbu)
            d_db = st(np.where(below > 0, dx, 0.0))
        # bottleneck (level L-1) and encoder
        d_e = d_db
        for l in range(L - 1, -1, -1):
            Wb, _ = self.weights(p, f"enc{l}b")
            dW, db_, dx = self.conv_bwd(A[f"ea{l}"], Wb, d_e)
            put(f"enc{l}b", dW, db_)
            d_ea = st(np.where(A[f"ea{l}"] > 0, dx, 0.0))
            Wa, _ = self.weights(p, f"enc{l}a")
            xin = A["x8"] if l == 0 else A[f"p{l - 1}"]
            dW, db_, dx = self.conv_bwd(xin, Wa, d_ea)
            put(f"enc{l}a", dW, db_)
            if l > 0:
                d_p = st(np.where(xin > 0, dx, 0.0))
                add = self.unpool_add(d_skip[l - 1], d_p, A[f"arg{l - 1}"], A[f"p{l - 1}"])
                summed = d_skip[l - 1] + add
                # the stored skip gradient receives the pooled gradient at each window's maximum, and the
                # sum is stored (rounded) again; elsewhere it is unchanged
                d_e = np.where(add != 0, st(summed), d_skip[l - 1])
        return loss, g

    @staticmethod
    def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        p = p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
        return p, m, v
