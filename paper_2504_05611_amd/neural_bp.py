"""Learned per-edge, per-iteration BP weights (neural BP), trained on sampled syndromes.

The forward and backward passes are the library's HIP kernels
(tmcs_wbp_forward / tmcs_wbp_backward); torch provides device memory, the loss
on the observables and the optimizer.

Loss (the paper does not train decoders; this is the library's reading): for
every iteration t and logical observable o, binary cross-entropy between the
observable flip o and the probability the BP marginals assign to it,
  P_t(o) = (1 - prod_{v in supp L_o} tanh(L_t(v) / 2)) / 2,
summed over t so that early iterations are pushed towards the answer too.
The product is evaluated in the log domain with sign tracking.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import tmcs


class WeightedBP(torch.autograd.Function):
    """L_all[T, S, n] = weighted min-sum posteriors after every iteration."""

    @staticmethod
    def forward(ctx, weights, det, dem, n_shots):
        T = weights.shape[0]
        n = dem.cols
        ws = torch.empty(dem.wbp_workspace_size(T, n_shots), dtype=torch.uint8, device=weights.device)
        llr = torch.empty((T, n_shots, n), dtype=torch.float32, device=weights.device)
        w = weights.detach().contiguous()
        dem.wbp_forward(w, T, det, n_shots, llr, ws)
        ctx.save_for_backward(w)
        ctx.dem, ctx.det, ctx.ws, ctx.n_shots = dem, det, ws, n_shots
        return llr

    @staticmethod
    def backward(ctx, grad_llr):
        (w,) = ctx.saved_tensors
        T = w.shape[0]
        gw = torch.zeros_like(w)
        ctx.dem.wbp_backward(w, T, ctx.det, ctx.n_shots, grad_llr.contiguous(), gw, ctx.ws)
        return gw, None, None, None


def observable_support(dem) -> torch.Tensor:
    """[k, n] 0/1 matrix of the columns that flip each observable."""
    L = dem.L().astype(np.float32)
    if L.shape[0] == 0:
        L = np.zeros((1, dem.cols), dtype=np.float32)
    return torch.from_numpy(L)


def observable_loss(llr, obs_bits, supp):
    """Sum over t and o of BCE(P_t(o), obs).  llr [T, S, n]; obs_bits [S, k] float; supp [k, n]."""
    a = llr.abs().clamp_min(1e-6)
    # log|tanh(L/2)|, kept finite so that columns outside supp(L_o) (weight 0) never give 0 * inf
    logt = (torch.log1p(-torch.exp(-a)) - torch.log1p(torch.exp(-a))).clamp_min(-60.0)
    neg = (llr < 0).to(llr.dtype)
    S_log = torch.einsum("tsn,kn->tsk", logt, supp)                      # log|prod tanh|
    parity = torch.remainder(torch.einsum("tsn,kn->tsk", neg, supp), 2.0)  # sign of the product
    e = torch.exp(S_log)
    # P(o = 1) = (1 - prod)/2, P(o = 0) = (1 + prod)/2, prod = (-1)^parity e^S_log
    one_minus = torch.where(parity > 0.5, 1.0 + e, -torch.expm1(S_log))
    one_plus = torch.where(parity > 0.5, -torch.expm1(S_log), 1.0 + e)
    log_p1 = torch.log(one_minus.clamp_min(1e-30)) - math.log(2.0)
    log_p0 = torch.log(one_plus.clamp_min(1e-30)) - math.log(2.0)
    y = obs_bits[None]
    return -(y * log_p1 + (1.0 - y) * log_p0).sum()


def weights_name(spec, T) -> str:
    """File stem under paper_2504_05611_amd/weights/ of the weights learned for a
    circuit (code, operation, noise, rounds) and T iterations."""
    code = "sc%d" % spec.d if spec.code == "sc" else spec.bb
    return "%s_%s_p%g_pe%g_r%d-%d_T%d" % (code, spec.op, spec.p, spec.p_ebit, spec.rounds_before,
                                          spec.rounds_after, T)


def save_weights(path, weights, train_syndromes, losses, extra=None):
    """[T, edges] weights, stored in FP16 (the decoder reads them as FP32: callers
    round with round_fp16 first and use the rounded values), plus what they were
    trained on (npz, no pickles)."""
    arrs = dict(weights=weights.detach().half().cpu().numpy(), train_syndromes=np.int64(train_syndromes),
                losses=np.asarray(losses, dtype=np.float32))
    for k, v in (extra or {}).items():
        arrs[k] = np.asarray(v)
    np.savez_compressed(path, **arrs)


def round_fp16(weights):
    """The weights as stored: rounded to FP16, back in FP32."""
    return weights.detach().half().float()


@dataclass
class TrainResult:
    weights: torch.Tensor
    losses: list


def unpack_obs(obs_words, n_shots, k):
    """[k, words] int64 bit planes -> [n_shots, k] float32 on the same device."""
    sh = torch.arange(64, device=obs_words.device, dtype=torch.int64)
    bits = (obs_words[:k, :, None] >> sh) & 1
    return bits.reshape(k, -1)[:, :n_shots].T.to(torch.float32)


def train(circuit, dem, T, *, steps=200, batch=256, lr=0.01, seed=2, init=1.0, log_every=0, last=0):
    """Train weights [T, E] on fresh syndromes sampled by the library each step.

    last > 0 restricts the loss to the last `last` iterations (all T otherwise).
    """
    dev = torch.device("cuda")
    w = torch.full((T, dem.edges), float(init), dtype=torch.float32, device=dev, requires_grad=True)
    opt = torch.optim.Adam([w], lr=lr)
    supp = observable_support(dem).to(dev)
    k = max(circuit.num_observables, 1)
    det, obs = circuit.alloc_outputs(batch)
    losses = []
    for step in range(steps):
        circuit.sample(seed, 0, step * ((batch + 4095) // 4096) * 4096, batch, det, obs)
        llr = WeightedBP.apply(w, det, dem, batch)
        y = unpack_obs(obs, batch, k)
        tl = llr[T - last:] if 0 < last < T else llr
        loss = observable_loss(tl, y, supp) / (batch * tl.shape[0])
        opt.zero_grad()
        loss.backward()
        opt.step()
        with torch.no_grad():
            w.clamp_(0.0, 4.0)
        losses.append(float(loss.detach()))
        if log_every and step % log_every == 0:
            print(f"step {step} loss {losses[-1]:.5f}", flush=True)
    return TrainResult(w.detach(), losses)


def evaluate(circuit, dem, *, n_shots, T, weights=None, alpha=1.0, use_osd=True, seed=11):
    """LER and OSD rate of (weighted) BP-OSD on fresh shots."""
    det, obs = circuit.alloc_outputs(n_shots)
    circuit.sample(seed, 0, 0, n_shots, det, obs)
    pred = torch.zeros_like(obs)
    st = tmcs.new_stats()
    dem.decode(det, n_shots, pred, max_iter=T, alpha=alpha, weights=weights, use_osd=use_osd, stats=st)
    ne, ler, sig = tmcs.logical_error_rate(pred, obs, circuit.num_observables, n_shots)
    s = tmcs.read_stats(st)
    return dict(errors=ne, ler=ler, sigma=sig, osd_rate=s["osd"] / max(n_shots, 1),
                converged=s["converged"] / max(n_shots, 1), bp_iters=s["bp_iters"] / max(n_shots, 1))


def main(argv=None):
    """Train weights on one workload's syndromes and compare learned with plain BP-OSD.

    Prints one JSON line: training throughput, loss trace summary, and for plain
    (alpha = 1) and learned weights the LER, OSD rate and BP convergence rate on
    the same fresh shots.
    """
    import argparse
    import json
    import time

    from workloads import WORKLOADS

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--workload", default="bb144_teleport")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=0.01)
    ap.add_argument("--last", type=int, default=0, help="loss over the last N iterations only (0: all)")
    ap.add_argument("--eval-shots", type=int, default=1 << 20)
    ap.add_argument("--out", default="", help="save the trained weights (.npz); 'auto' writes "
                                             "paper_2504_05611_amd/weights/<circuit>_T<T>.npz")
    ap.add_argument("--log-every", type=int, default=20)
    ap.add_argument("--d", type=int, default=0, help="pick the workload's circuit of this distance")
    ap.add_argument("--p", type=float, default=0.0, help="pick the workload's circuit of this p")
    args = ap.parse_args(argv)
    w = WORKLOADS[args.workload]
    spec = next(s for s in w.specs if (not args.d or s.d == args.d) and (not args.p or s.p == args.p))
    T = w.bp_iters
    circuit = tmcs.Circuit(spec)
    dem = tmcs.DEM(circuit)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = train(circuit, dem, T, steps=args.steps, batch=args.batch, lr=args.lr, seed=w.seed + 1,
                log_every=args.log_every, last=args.last)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    res.weights = round_fp16(res.weights)       # the stored (and evaluated) weights
    if args.out:
        import os
        out_path = args.out
        if out_path == "auto":
            wdir = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
            os.makedirs(wdir, exist_ok=True)
            out_path = os.path.join(wdir, weights_name(spec, T) + ".npz")
        elif os.path.isdir(out_path):
            out_path = os.path.join(out_path, weights_name(spec, T) + ".npz")
        save_weights(out_path, res.weights, args.steps * args.batch, res.losses,
                     dict(lr=args.lr, batch=args.batch, steps=args.steps, loss_iterations=args.last or T))
    out = dict(workload=w.name, d=spec.d, p=spec.p, T=T, edges=dem.edges, train_steps=args.steps, batch=args.batch, lr=args.lr,
               loss_iterations=args.last or T,
               train_syndromes=args.steps * args.batch, train_s=t_train,
               train_syndromes_per_s=args.steps * args.batch / t_train,
               loss_first=float(np.mean(res.losses[: max(1, len(res.losses) // 10)])),
               loss_last=float(np.mean(res.losses[-max(1, len(res.losses) // 10):])))
    for name, wts in (("plain", None), ("learned", res.weights)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = evaluate(circuit, dem, n_shots=args.eval_shots, T=T, weights=wts, seed=w.seed)
        torch.cuda.synchronize()
        r["decode_s"] = time.perf_counter() - t1
        out[name] = r
    print(json.dumps(out))


if __name__ == "__main__":
    main()
