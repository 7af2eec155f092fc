"""The learned slice-map surrogate (include/nv_surrogate.h) over torch device
memory.

Argument marshalling only: training, inference, the training-set gather and
the composition run in libnv's HIP kernels.  torch provides the device buffers
and the stream.
"""
from __future__ import annotations

import numpy as np

from . import nv
from .propagator import Batch, Propagator
from .workloads import SUR_IN_SCALE, SUR_IN_SHIFT, SUR_OUT_SCALE, SUR_SLICE_LENGTH


class Surrogate:
    """correction "additive" (phi ~ G + out_scale * out) or "step-doubling"
    (phi ~ G1 + d (16/15 + out_scale g out), gate and loss_scale per component);
    see include/nv_surrogate.h."""

    def __init__(self, device="cuda:0", max_batch=65536, in_shift=SUR_IN_SHIFT,
                 in_scale=SUR_IN_SCALE, out_scale=SUR_OUT_SCALE, slice_length=SUR_SLICE_LENGTH,
                 coarse_steps=0, stream=None, correction="additive", gate=(1.0, 1.0),
                 loss_scale=(1.0, 1.0)):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("Surrogate needs a GPU device")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.in_shift, self.in_scale = tuple(in_shift), tuple(in_scale)
        self.out_scale = tuple(out_scale)
        self.slice_length, self.coarse_steps = float(slice_length), int(coarse_steps)
        self.max_batch = int(max_batch)
        self.correction = correction
        self.target_rows = 4 if correction == "step-doubling" else 2
        self._visits = None
        kind = {"additive": nv.NV_SUR_ADDITIVE, "step-doubling": nv.NV_SUR_STEP_DOUBLING}
        with torch.cuda.device(self.device):
            cfg = nv.make_sur_config(in_shift, in_scale, out_scale, slice_length, coarse_steps,
                                     max_batch, self.stream.cuda_stream, kind[correction], gate,
                                     loss_scale)
            self.h = nv.nv_sur_create(cfg)

    def close(self):
        if getattr(self, "h", None) is not None:
            nv.nv_sur_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- parameters -----------------------------------------------------------
    def set_params(self, params):
        nv.nv_sur_set_params(self.h, params)

    def params(self) -> np.ndarray:
        return nv.nv_sur_get_params(self.h)

    # -- data -------------------------------------------------------------------
    def _dev(self, a, dtype):
        t = self.torch
        a = a if isinstance(a, t.Tensor) else t.from_numpy(np.ascontiguousarray(a))
        return a.to(device=self.device, dtype=dtype).contiguous()

    def forward(self, x):
        """x: (4, n) raw inputs -> (2, n) network outputs (device tensors)."""
        x = self._dev(x, self.torch.float32)
        n = x.shape[1]
        out = self.torch.empty((2, n), dtype=self.torch.float32, device=self.device)
        self.stream.synchronize()
        nv.nv_sur_forward(self.h, x.data_ptr(), n, out.data_ptr())
        return out

    def loss_grad(self, x, target):
        """Mean loss and flat gradient (numpy fp32) of one minibatch."""
        x = self._dev(x, self.torch.float32)
        target = self._dev(target, self.torch.float32)
        self.stream.synchronize()
        return nv.nv_sur_loss_grad(self.h, x.data_ptr(), target.data_ptr(), x.shape[1])

    def train(self, x, target, batch, steps, lr=1e-3, lr_final=0.0, beta1=0.9, beta2=0.999,
              eps=1e-8):
        """Adam steps over a device data set; returns the per-step losses (device)."""
        x = self._dev(x, self.torch.float32)
        target = self._dev(target, self.torch.float32)
        losses = self.torch.empty(int(steps), dtype=self.torch.float32, device=self.device)
        self.stream.synchronize()
        nv.nv_sur_train(self.h, x.data_ptr(), target.data_ptr(), x.shape[1],
                        nv.make_train_opts(batch, steps, lr, beta1, beta2, eps, lr_final),
                        losses.data_ptr() if steps > 0 else None)
        return losses

    def dataset_from_batch(self, batch: Batch, perm=None):
        """(x (4, n), target (2, n)) device tensors from the tables of a run batch;
        sample number i goes to column perm[i]."""
        t = self.torch
        total = nv.nv_sur_dataset_from_batch(self.h, batch.batch)
        x = t.empty((4, total), dtype=t.float32, device=self.device)
        tg = t.empty((self.target_rows, total), dtype=t.float32, device=self.device)
        p = None
        if perm is not None:
            p = self._dev(perm, t.int64)
            if p.numel() != total:
                raise ValueError(f"perm has {p.numel()} entries, the batch {total} samples")
        self.stream.synchronize()
        nv.nv_sur_dataset_from_batch(self.h, batch.batch, p.data_ptr() if p is not None else None,
                                     x.data_ptr(), tg.data_ptr(), total)
        return x, tg

    def set_visits(self, states, mu_lo, mu_hi, sigma, floor_weight):
        """Visit weights of the step-doubling training set from chains of states,
        (n_mu, n_states, 2) FP64 (a device tensor is kept alive here); None
        switches them off."""
        t = self.torch
        if states is None:
            nv.nv_sur_set_visits(self.h, None, 0, 0, 0.0, 0.0, 0.0, 0.0)
            self._visits = None
            return
        st = self._dev(states, t.float64).contiguous()
        if st.dim() != 3 or st.shape[2] != 2:
            raise ValueError("states must be (n_mu, n_states, 2)")
        self.stream.synchronize()
        nv.nv_sur_set_visits(self.h, st.data_ptr(), st.shape[0], st.shape[1], mu_lo, mu_hi,
                             sigma, floor_weight)
        self._visits = st

    # -- the composition ------------------------------------------------------------
    def compose(self, y0, mu, t0, T, n_slices, fallback: Propagator | None = None, guard=0.0,
                box_lo=(-3.0, -8.0), box_hi=(3.0, 8.0), want_boundary=False):
        """Chains q = 0..count-1 from y0[q] with parameter mu[q].  Returns (status,
        final (count, 2), boundary (count, N+1, 2) or None, info), device tensors."""
        t = self.torch
        y0 = self._dev(np.asarray(y0, np.float64).reshape(-1, 2)
                       if not isinstance(y0, t.Tensor) else y0, t.float64).reshape(-1, 2)
        count = y0.shape[0]
        mu = self._dev(np.asarray(mu, np.float64).reshape(-1)
                       if not isinstance(mu, t.Tensor) else mu, t.float64).reshape(-1)
        if mu.numel() != count:
            raise ValueError("one mu per chain")
        final = t.empty((count, 2), dtype=t.float64, device=self.device)
        bnd = (t.empty((count, n_slices + 1, 2), dtype=t.float64, device=self.device)
               if want_boundary else None)
        c = nv.nv_sur_chains()
        c.count, c.y0, c.mu = count, y0.data_ptr(), mu.data_ptr()
        c.t0, c.T, c.n_slices = float(t0), float(T), int(n_slices)
        c.final_state = final.data_ptr()
        c.boundary = bnd.data_ptr() if bnd is not None else None
        c.guard = float(guard)
        for k in range(2):
            c.box_lo[k], c.box_hi[k] = float(box_lo[k]), float(box_hi[k])
        if fallback is not None:
            w = fallback.workload
            if (w is None or w.rhs != "vdp" or w.interp != "bilinear" or w.n_slices != n_slices
                    or w.t0 != t0 or w.T != T):
                raise ValueError("the fallback must be a built Van der Pol context with the "
                                 "same interval and slices")
            if not bool((mu == float(w.params[0])).all()):
                raise ValueError("every chain must have the fallback table's mu")
            c.fb_tab0 = nv.nv_table_device_ptr(fallback.ctx, 0)
            c.fb_tab1 = nv.nv_table_device_ptr(fallback.ctx, 1)
            c.fb_precision = nv.PRECISIONS[w.precision]
            c.fb_grid = Propagator.grid(w)
            fallback.stream.synchronize()
        self.stream.synchronize()
        st, info = nv.nv_sur_compose(self.h, c)
        return st, final, bnd, info

    def last_ms(self) -> float:
        return nv.nv_sur_last_ms(self.h)
