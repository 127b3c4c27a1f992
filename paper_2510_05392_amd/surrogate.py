"""Surrogate-assisted unweighting on top of the exact matrix element.

Orchestration only (argument marshalling and loops): the features, the
network's forward and backward passes, Adam, the exact matrix elements and
both unweighting stages run in the HIP kernels of libmegpu.so; torch tensors
only hold device memory.

  fit()       labels events with the exact FP64 path, normalises the features
              (pair invariants) and the targets (log|M|^2), trains the MLP with
              minibatch Adam on the GPU;
  predict()   normalised log|M|^2 from the network;
  unweight()  two-stage unweighting (Danziger et al., SciPost Phys. 12 (2022) 164):
              stage 1 on the surrogate weight, stage 2 corrects the accepted
              events with the exact matrix element; plus the one-stage
              reference that needs the exact weight of every event.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import binding


class SurrogatePipeline:
    def __init__(self, process='gg_ttxgg', width=256, depth=4, seed=1, alpha_s=0.118,
                 colorsum_mode=binding.ME_CS_FP64):
        import torch
        self.torch = torch
        self.me = binding.MatrixElement(process, colorsum_mode=colorsum_mode)
        self.npar = self.me.npar
        self.nfeat = self.npar * (self.npar - 1) // 2
        self.sur = binding.Surrogate(self.nfeat, width, depth, seed)
        self.alpha_s = alpha_s
        self.dev = torch.device('cuda:0')
        self.ymean = 0.0
        self.ystd = 1.0

    # ---------------------------------------------------------------- helpers
    def _empty(self, shape, dtype):
        return self.torch.empty(shape, dtype=dtype, device=self.dev)

    def exact(self, mom):
        """Exact |M|^2 (device float64) of device momenta [n][npar][4]."""
        out = self._empty(mom.shape[0], self.torch.float64)
        self.me.me_compute(mom, mom.shape[0], self.alpha_s, out, self.torch.cuda.current_stream())
        return out

    def features(self, mom, raw=False):
        n = mom.shape[0]
        feat = self._empty((n, self.sur.kpad), self.torch.int16)
        rawt = self._empty((n, self.nfeat), self.torch.float32) if raw else None
        self.sur.me_sur_features(mom, n, self.npar, feat, rawt, self.torch.cuda.current_stream())
        return (feat, rawt) if raw else feat

    # ---------------------------------------------------------------- training
    def fit(self, mom, epochs=20, batch=4096, lr=2e-3, lr_final=1e-4, seed=0, log=None):
        """Train on device momenta; returns the per-epoch mean training losses.

        Labels come from the exact FP64 path; normalisation statistics, targets and
        each epoch's shuffled copy of the training set are formed by library
        kernels (the permutation is drawn on the host and passed in)."""
        torch = self.torch
        n = mom.shape[0]
        stream = torch.cuda.current_stream()
        me2 = self.exact(mom)
        _, raw = self.features(mom, raw=True)
        self.ymean, self.ystd = self.sur.me_sur_fit_normalisation(raw, n, me2, stream)
        feat = self.features(mom)
        target = self._empty(n, torch.float32)
        binding.me_sur_targets(me2, n, self.ymean, self.ystd, target, stream)
        rng = np.random.Generator(np.random.PCG64(seed))
        nbatch = n // batch
        loss = torch.zeros(1, dtype=torch.float32, device=self.dev)
        fe = self._empty(feat.shape, feat.dtype)
        ta = self._empty(n, torch.float32)
        history = []
        step = 0
        total_steps = epochs * nbatch
        for ep in range(epochs):
            perm = torch.from_numpy(rng.permutation(n).astype(np.int64)).to(self.dev)
            binding.me_sur_gather_rows(feat, target, perm, n, self.sur.kpad, fe, ta, stream)
            loss.zero_()
            for b in range(nbatch):
                # cosine decay from lr to lr_final
                frac = step / max(1, total_steps - 1)
                lr_now = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * frac))
                self.sur.me_sur_train_step(fe[b * batch:(b + 1) * batch], ta[b * batch:(b + 1) * batch], batch,
                                           lr_now, loss, stream)
                step += 1
            history.append(float(loss.item()) / (nbatch * batch))
            if log:
                log(f'epoch {ep}: mse {history[-1]:.4e}')
        return history

    def predict(self, mom=None, feat=None):
        """Normalised network output (float32 device tensor)."""
        if feat is None:
            feat = self.features(mom)
        n = feat.shape[0]
        y = self._empty(n, self.torch.float32)
        self.sur.me_sur_predict(feat, n, y, self.torch.cuda.current_stream())
        return y

    def log_error(self, mom):
        """(RMS, largest absolute) error of the surrogate's log|M|^2 on these events."""
        y = self.predict(mom)
        return binding.me_sur_log_error(y, self.exact(mom), mom.shape[0], self.ymean, self.ystd,
                                        self.torch.cuda.current_stream())

    # ---------------------------------------------------------------- unweighting
    def calibrate(self, mom, wps, quantile=1.0):
        """Maxima (or q-quantiles) of the surrogate weight and of the exact/surrogate
        ratio on a calibration sample."""
        y = self.predict(mom)
        return binding.me_unweight_maxima(y, wps, self.exact(mom), mom.shape[0], self.ymean, self.ystd, quantile,
                                          self.torch.cuda.current_stream())

    def exact_weight_max(self, mom, wps, quantile=1.0):
        """Maximum (or q-quantile) of the exact weights |M|^2 wps, for one-stage unweighting."""
        return binding.me_unweight_quantile(self.exact(mom), wps, mom.shape[0], quantile,
                                            self.torch.cuda.current_stream())

    @staticmethod
    def _summary(res, resid, m):
        acc, over, sw, sw2 = binding.me_unweight_summary(resid, m)
        res.update({'accepted': acc, 'overweight': over, 'sum_w': sw, 'sum_w2': sw2,
                    'ess': (sw * sw / sw2) if sw2 > 0 else 0.0})
        return res

    def unweight(self, mom, wps, r1, r2, what_max, x_max):
        """Two-stage unweighting of device momenta; returns a dict of results and timings:
        'index' (stage-1 event indices) and 'resid' (their residual weights, 0 where
        stage 2 rejected) as device tensors, counts, weight sums and the Kish
        effective sample size of the accepted sample."""
        torch = self.torch
        n = mom.shape[0]
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        feat = self.features(mom)
        y = self.predict(feat=feat)
        what = self._empty(n, torch.float64)
        idx = self._empty(n, torch.int64)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        m = binding.me_unweight_stage1(y, wps, r1, n, self.ymean, self.ystd, what_max, what, idx, stream)
        sel = self._empty((max(m, 1), self.npar, 4), torch.float64)
        binding.me_gather_momenta(mom, idx, m, self.npar, sel, stream)
        me_sel = self.exact(sel[:m]) if m else self._empty(0, torch.float64)
        resid = self._empty(max(m, 1), torch.float64)
        binding.me_unweight_stage2(me_sel, idx, m, wps, what, r2, what_max, x_max, resid, stream)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res = {'n': n, 'stage1': m, 'index': idx[:m], 'resid': resid[:m], 'time_surrogate': t1 - t0,
               'time_total': t2 - t0}
        return self._summary(res, resid, m)

    def unweight_exact(self, mom, wps, r, w_max):
        """One-stage reference: exact weight of every event, accept with min(1, w / w_max);
        'resid' holds every event's residual weight (0 = rejected)."""
        torch = self.torch
        n = mom.shape[0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        resid = self._empty(n, torch.float64)
        binding.me_unweight_onestage(self.exact(mom), wps, r, n, w_max, resid, torch.cuda.current_stream())
        torch.cuda.synchronize()
        res = {'n': n, 'resid': resid, 'time_total': time.perf_counter() - t0}
        return self._summary(res, resid, n)
