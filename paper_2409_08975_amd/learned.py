"""Learned importance proposal over the C ABI (an extension of the paper's
sampler).

The method samples the centre edge p of a delta-centred 3-path with
probability w_p / W.  Here a small network g(f_p) over per-edge window
features is trained on closure outcomes of the method's own samples (drawn
on a Philox stream that no estimate uses), turned into integer factors
h_p = max(1, round((eps + (1 - eps) g) 2^s)), and the centre edge is drawn
with probability w_p h_p / Q.  Each sample is corrected by Q / h_p, so the
estimate stays unbiased whatever the network learned; a pilot run compares
the per-sample variance against the method's and keeps the method when the
proposal does not help.  Every step runs in libtc.so kernels; this module
only sequences the calls and does scalar bookkeeping on the host.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import (MLP_PARAMS, Graph, Weights, new_result, tc_edge_features, tc_mlp_forward,
               tc_mlp_train, tc_proposal_weights, tc_proposal_window, tc_quantize_proposal,
               tc_sample_estimate, tc_window_factors)

LABEL_STREAM = 0x4C000000  # Philox stream of the training labels


def init_params(seed: int, base_rate: float = 0.5) -> np.ndarray:
    """He-normal weight matrices, zero biases, output bias at the logit of
    the label base rate (float32, the parameter order of the C ABI)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(MLP_PARAMS, np.float32)
    o = 0
    p[o:o + 512] = rng.standard_normal(512) * math.sqrt(2.0 / 8)
    o += 512 + 64
    p[o:o + 4096] = rng.standard_normal(4096) * math.sqrt(2.0 / 64)
    o += 4096 + 64
    p[o:o + 64] = rng.standard_normal(64) * math.sqrt(1.0 / 64)
    r = min(max(base_rate, 1e-6), 1 - 1e-6)
    p[MLP_PARAMS - 1] = math.log(r / (1 - r))
    return p


@dataclass
class Moments:
    """Mean and variance of one run's per-sample estimator."""
    estimate: float
    var: float  # per-sample variance of X W (plain) or X Q / h (proposal)
    k: int

    @property
    def stderr(self) -> float:
        return math.sqrt(max(self.var, 0.0) / self.k)


def moments(result, weights: Weights, k: int, j: int = 0) -> Moments:
    """Per-sample variance from cnt and the second moment m2 (host scalars)."""
    total = int(weights.view("S", torch.int64, weights.c.m + 1)[-1].item()) & (2**64 - 1)
    cnt = result.counts()[j]
    m2 = float(result.m2[j].item())
    # a proposal set (centre or window factors) accumulates floor(X 2^64 / h)
    mean_x = cnt / k if weights.base is None else cnt / 2.0**64 / k
    var = total * total * (m2 / k - mean_x * mean_x)
    return Moments(float(result.estimate[j].item()), var, k)


class LearnedProposal:
    def __init__(self, graph: Graph, weights: Weights, motif, eps: float = 0.01, seed: int = 1,
                 normalize: bool = True):
        self.graph, self.weights, self.motif = graph, weights, motif
        self.eps, self.seed, self.normalize = eps, seed, normalize
        self.feat = tc_edge_features(graph, weights)
        self.params = None
        self.opt = None
        self.losses = None
        self.proposal: Weights | None = None

    def collect_labels(self, n_labels: int):
        """Closure outcomes of n_labels samples of the method (per-sample X
        and the centre positions P) on the label stream."""
        r = tc_sample_estimate(self.graph, self.weights, [self.motif], n_labels, self.seed,
                               stream_id=LABEL_STREAM, per_sample=True)
        return r

    def fit(self, n_labels: int = 10**6, epochs: int = 8, batch: int = 8192, lr: float = 3e-3,
            label_cap: float = 64.0):
        """Train on closure outcomes: y = [X > 0], or min(1, X / label_cap)."""
        lab = self.collect_labels(n_labels)
        rate = int(lab.hits[0].item()) / n_labels
        if label_cap > 0:  # mean soft label, roughly
            rate = min(rate, lab.counts()[0] / n_labels / label_cap)
        dev = self.feat.device
        self.params = torch.from_numpy(init_params(self.seed, max(rate, 1e-4))).to(dev)
        self.opt = torch.zeros(2 * MLP_PARAMS, dtype=torch.float32, device=dev)
        X = lab.X[0]
        self.losses = tc_mlp_train(self.params, self.opt, self.feat, lab.P, X, batch, epochs, lr,
                                   self.seed, label_cap=label_cap)
        self.label_rate = rate
        return self.losses

    def build_proposal(self) -> Weights:
        g = tc_mlp_forward(self.params, self.feat)
        h = tc_quantize_proposal(self.weights, g, self.eps, normalize=self.normalize)
        self.proposal = tc_proposal_weights(self.graph, self.weights, h)
        return self.proposal

    def pilot(self, k: int, seed: int):
        """(method's Moments, proposal's Moments) from one pilot run each."""
        rp = tc_sample_estimate(self.graph, self.weights, [self.motif], k, seed, moments=True)
        ri = tc_sample_estimate(self.graph, self.proposal, [self.motif], k, seed, moments=True)
        return moments(rp, self.weights, k), moments(ri, self.proposal, k)

    def choose(self, k_pilot: int = 10**6, seed: int = 0x5EED):
        """The weight set to estimate with: the proposal unless its pilot
        variance exceeds the method's."""
        mp, mi = self.pilot(k_pilot, seed)
        self.pilot_ratio = mp.var / mi.var if mi.var > 0 else float("inf")
        return self.proposal if mi.var <= mp.var else self.weights


class WindowProposal:
    """Importance sampling over the side edges as well (tc_proposal_window):
    every CSR entry carries the factor min(cap, (1 + degree of its far
    endpoint)^(quarter / 4)) in integer square roots, each side's edge is
    drawn by factor and the centre edge by h_p G1_p G3_p.  The heavy closure
    counts of a path come from hub endpoints inside its windows, which a
    factor on the centre edge alone cannot single out.  The exponent and the
    cap are chosen from pilot runs (the lowest measured per-sample variance
    among the candidates whose total fits 64 bits); an optional centre factor
    h (from LearnedProposal) multiplies in."""

    CANDIDATES = ((1, 65535), (2, 65535), (3, 65535), (2, 255), (3, 255))

    def __init__(self, graph: Graph, weights: Weights, motif, h: torch.Tensor | None = None):
        self.graph, self.weights, self.motif, self.h = graph, weights, motif, h
        self.proposal: Weights | None = None
        self.choice = None
        self.trials = []

    def build(self, quarter: int, cap: int) -> Weights:
        f_in, f_out = tc_window_factors(self.graph, quarter, cap)
        self.proposal = tc_proposal_window(self.graph, self.weights, self.h, f_in, f_out)
        return self.proposal

    def pilot(self, k: int, seed: int, stream_id: int = 0):
        rp = tc_sample_estimate(self.graph, self.weights, [self.motif], k, seed,
                                stream_id=stream_id, moments=True)
        rw = tc_sample_estimate(self.graph, self.proposal, [self.motif], k, seed,
                                stream_id=stream_id, moments=True)
        return moments(rp, self.weights, k), moments(rw, self.proposal, k)

    def fit(self, k_pilot: int = 10**6, seed: int = 0x5EED, candidates=None):
        """Pick (quarter, cap) by pilot variance on the label stream."""
        best = None
        self.trials = []
        for quarter, cap in candidates or self.CANDIDATES:
            self.build(quarter, cap)
            if self.proposal.status() != 0:  # total beyond 64 bits
                self.trials.append((quarter, cap, None))
                continue
            r = tc_sample_estimate(self.graph, self.proposal, [self.motif], k_pilot, seed,
                                   stream_id=LABEL_STREAM, moments=True)
            if int(r.status.item()) & 0xFFFFFFFF:
                self.trials.append((quarter, cap, None))
                continue
            v = moments(r, self.proposal, k_pilot).var
            self.trials.append((quarter, cap, v))
            if best is None or v < best[2]:
                best = (quarter, cap, v)
        if best is None:
            self.proposal = None
            return None
        self.choice = best[:2]
        return self.build(*self.choice)
