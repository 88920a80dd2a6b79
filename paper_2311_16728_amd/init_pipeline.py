"""Training data, training and evaluation of the learned initialiser.

Section 3.3.1 adds temporary primitives at inactive keypoints of a new
keyframe, placed at the keypoint's depth.  Here a keypoint is synthetic: a
visible Gaussian of a seeded room scene is held out of the map, and its
projected centre, camera depth and footprint octave form the keypoint.  The
map without the held-out Gaussians (the converged map a new keyframe meets;
optionally perturbed) plus the new primitives is optimised for a fixed number of batched mapping
iterations over every keyframe and pyramid level; the converged parameters of
the new primitives, relative to the heuristic start (log-scale and colour as
corrections, rotation in the keyframe's camera frame), are the labels and the
keyframe's 7x7 patch around the keypoint (with the keypoint's depth, scale and
the heuristic's log-scale) is the input.

Evaluation repeats the construction on held-out seeds and compares the
photometric loss (Eq. 4 summed over the pyramid, Eq. 5) after the same number
of iterations when the new primitives start from the heuristic and from the
network (heuristic fallback where the predicted opacity is below 0.01).

Run as a module:  python -m paper_2311_16728_amd.init_pipeline [--quick]
"""

from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np
import torch

import scenes
from . import gs
from .batching import BatchedMapper
from .init_mlp import N_IN_PAD, N_TARGET, InitMLP
from .mapper import LAMBDA, PYRAMID_LEVELS, RenderPlan, mapping_lr_rows

C0 = 0.28209479177387814          # degree-0 real SH value
OCTAVE_BASE_PX = 2.0              # footprint radius of octave 0 (pixels)


def _quat_mul(a, b):
    w1, x1, y1, z1 = a.unbind(-1)
    w2, x2, y2, z2 = b.unbind(-1)
    return torch.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                        w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], -1)


def _mat_to_quat(R: np.ndarray) -> np.ndarray:
    from scipy.spatial.transform import Rotation
    x, y, z, w = Rotation.from_matrix(np.asarray(R, np.float64)).as_quat()
    return np.array([w, x, y, z])


class Case:
    """One seeded scene with held-out keypoints in each keyframe."""

    def __init__(self, seed: int, n: int = 500_000, n_kf: int = 8, per_kf: int = 4096,
                 width: int = 1200, height: int = 680, f: float = 600.0, perturb_map: bool = False,
                 kf_stride: int = 10, min_weight: float = 0.1, device="cuda"):
        self.seed, self.device = seed, device
        gt, pert, cams = scenes.room_scene(seed, n, n_kf, width, height, f, kf_stride=kf_stride)
        self.cams = cams
        rng = np.random.default_rng(seed + 104729)
        Pgt = torch.as_tensor(gt).to(device)
        # ground-truth images and per-Gaussian visible weight sum_pixels alpha*T in each keyframe
        plan = RenderPlan(cams, [(v, 0, (0, 0, 0), 1.0) for v in range(n_kf)], gt.shape[1], 1 << 27)
        plan.render(Pgt, n)
        if plan.overflowed():
            raise RuntimeError("pair buffer overflow while rendering the ground truth")
        self.gt_images = [plan.image(plan.rgb, v).clone() for v in range(n_kf)]
        taken = np.zeros(n, bool)
        self.held = []            # per keyframe: GT column indices
        self.kp = []              # per keyframe: [B][4] float32 (u, v, depth, scale)
        for v, cam in enumerate(cams):
            one = RenderPlan([cam], [(0, 0, (0, 0, 0), 1.0)], gt.shape[1], 1 << 25)
            one.render(Pgt, n)
            dL = torch.zeros(3 * one.total_pixels, dtype=torch.float32, device=device)
            dL[:one.total_pixels] = 1.0
            grad = torch.zeros_like(Pgt)
            one.backward(Pgt, n, dL, grad)
            if one.overflowed():
                raise RuntimeError("pair buffer overflow while scoring visibility")
            weight = (grad[11, :n] / C0).cpu().numpy()
            R = np.asarray(cam["R"], np.float64)
            xc = gt[0:3, :n].T.astype(np.float64) @ R.T + np.asarray(cam["t"], np.float64)
            z = xc[:, 2]
            u = cam["fx"] * xc[:, 0] / np.maximum(z, 1e-9) + cam["cx"]
            vv = cam["fy"] * xc[:, 1] / np.maximum(z, 1e-9) + cam["cy"]
            ok = ((weight >= min_weight) & (z > 0.3) & (u >= 4) & (u < width - 4) & (vv >= 4) &
                  (vv < height - 4) & ~taken)
            cand = np.nonzero(ok)[0]
            pick = np.sort(rng.choice(cand, size=min(per_kf, cand.size), replace=False))
            taken[pick] = True
            r_px = cam["fx"] * np.exp(gt[3:6, pick].astype(np.float64).mean(axis=0)) / z[pick]
            octave = np.clip(np.rint(np.log(r_px / OCTAVE_BASE_PX) / math.log(1.2)), 0, 7)
            kp = np.stack([u[pick], vv[pick], z[pick], 1.2 ** octave], 1).astype(np.float32)
            self.held.append(pick)
            self.kp.append(kp)
        held_all = np.concatenate(self.held)
        keep = np.ones(n, bool)
        keep[held_all] = False
        self.n_exist = int(keep.sum())
        self.n_new = int(held_all.size)
        self.n_total = self.n_exist + self.n_new
        self.n_cap = scenes.pad_cap(self.n_total)
        base = np.zeros((59, self.n_cap), np.float32)
        # the map the new keyframe meets: converged (the ground truth) or perturbed
        base[:, :self.n_exist] = (pert if perturb_map else gt)[:, :n][:, keep]
        self.base = base
        self.gt_new = [gt[:, h] for h in self.held]

    # -- initialisation of the new primitives ---------------------------------
    def _heuristic(self, P, n_exist, v):
        kp = self.kp[v]
        cam = self.cams[v]
        R = np.asarray(cam["R"], np.float64)
        t = np.asarray(cam["t"], np.float64)
        xc = np.stack([kp[:, 2] * (kp[:, 0] - cam["cx"]) / cam["fx"],
                       kp[:, 2] * (kp[:, 1] - cam["cy"]) / cam["fy"], kp[:, 2]], 1).astype(np.float64)
        mu = (xc - t) @ R
        img = self.gt_images[v]
        ui = torch.as_tensor(np.rint(kp[:, 0]).astype(np.int64), device=self.device)
        vi = torch.as_tensor(np.rint(kp[:, 1]).astype(np.int64), device=self.device)
        rgb = img[:, vi.clamp(0, img.shape[1] - 1), ui.clamp(0, img.shape[2] - 1)].contiguous()
        out = torch.empty(59, kp.shape[0], dtype=torch.float32, device=self.device)
        gs.gs_init_heuristic(torch.as_tensor(mu.T.astype(np.float32)).to(self.device).contiguous(), rgb,
                             P, n_exist, out)
        return out

    def features(self, v, heur=None) -> torch.Tensor:
        kp = torch.as_tensor(self.kp[v]).to(self.device)
        x = torch.empty(kp.shape[0], N_IN_PAD, dtype=torch.int16, device=self.device)
        gs.gs_init_features(self.gt_images[v], kp, x, heur)
        return x

    def initial_params(self, net: InitMLP | None = None):
        """Parameter store with the new primitives appended.  Returns (P,
        fallback fraction, heuristic columns per keyframe)."""
        P = torch.as_tensor(self.base).to(self.device)
        n_cur, fallback, count, heurs = self.n_exist, 0, 0, []
        for v in range(len(self.cams)):
            heur = self._heuristic(P, self.n_exist, v)
            heurs.append(heur)
            new = heur
            if net is not None:
                y = net.forward(self.features(v, heur))
                new = torch.empty_like(heur)
                used = torch.zeros(heur.shape[1], dtype=torch.int32, device=self.device)
                gs.gs_init_decode(y, torch.as_tensor(self.kp[v]).to(self.device), gs.make_view(self.cams[v]),
                                  heur, new, used)
                fallback += int(used.sum())
            count += heur.shape[1]
            gs.gs_append(P, None, None, n_cur, new)
            n_cur += heur.shape[1]
        assert n_cur == self.n_total
        return P, fallback / max(count, 1), heurs

    def mapper(self, P, lr_rows=None):
        return BatchedMapper(P, self.n_total, self.cams, self.gt_images, PYRAMID_LEVELS,
                             lr_rows=mapping_lr_rows() if lr_rows is None else lr_rows)

    # -- labels ----------------------------------------------------------------
    def labels(self, P, heurs) -> list[torch.Tensor]:
        """Targets of the network for the new primitives per keyframe ([B][11]
        float32): log-scale minus the heuristic's, unit quaternion relative to
        the keyframe's camera (w >= 0), opacity logit, SH DC minus the
        heuristic's."""
        out, at = [], self.n_exist
        Pc = P.double().cpu()
        for v, cam in enumerate(self.cams):
            B = self.kp[v].shape[0]
            cols = Pc[:, at:at + B]
            h = heurs[v].double().cpu()
            at += B
            ls = (cols[3:6] - h[3:6]).T
            qw = cols[6:10].T
            qw = qw / qw.norm(dim=1, keepdim=True).clamp_min(1e-12)
            qr = torch.as_tensor(_mat_to_quat(cam["R"]))[None].expand_as(qw)
            qc = _quat_mul(qr, qw)
            qc = torch.where(qc[:, :1] < 0, -qc, qc)
            out.append(torch.cat([ls, qc, cols[10:11].T, (cols[11:14] - h[11:14]).T], 1).float())
        return out


def run(bm: BatchedMapper, iters: int, record: bool = False):
    hist = torch.zeros(iters + 1, dtype=torch.float32, device=bm.params.device)
    for i in range(iters):
        bm.iteration()
        if record:
            hist[i].copy_(bm.plan.d_total[0])
    final = final_loss(bm)
    hist[iters] = final
    return final, hist.cpu().numpy()


def final_loss(bm: BatchedMapper) -> float:
    bm.plan.render(bm.params, bm.n)
    bm.plan.loss(bm.target, bm.lam, False)
    return float(bm.plan.d_total.item())


def psnr_level0(bm: BatchedMapper) -> float:
    vals = []
    for v in range(bm.plan.n_views):
        i = v * bm.levels
        a = bm.plan.image(bm.plan.rgb, i).clamp(0, 1)
        b = bm.plan.image(bm.target, i).clamp(0, 1)
        vals.append(10 * math.log10(1.0 / max(float(((a - b) ** 2).mean()), 1e-12)))
    return float(np.mean(vals))


def generate(seeds, iters=100, log=print, **case_kw):
    """(features, labels, heuristic start) for every held-out keypoint of the
    seeds' scenes; labels and heuristic start in the keyframe's camera frame."""
    X, Y, H = [], [], []
    for s in seeds:
        t0 = time.time()
        c = Case(s, **case_kw)
        P, _, heurs = c.initial_params(None)
        H += [h.to(c.device) for h in c.labels(P, heurs)]
        bm = c.mapper(P)
        loss, _ = run(bm, iters)
        for v, lab in enumerate(c.labels(bm.params, heurs)):
            X.append(c.features(v, heurs[v]))
            Y.append(lab.to(c.device))
        if log:
            log(f"scene {s}: {c.n_new} pairs, loss after {iters} iterations {loss:.4f} ({time.time() - t0:.1f}s)")
        del c, bm, P
    return torch.cat(X), torch.cat(Y), torch.cat(H)


GROUPS = {"log_scale": slice(0, 3), "quat": slice(3, 7), "opacity_logit": slice(7, 8), "sh_dc": slice(8, 11)}


def param_errors(pred: torch.Tensor, label: torch.Tensor) -> dict:
    """Mean squared error per parameter group (camera frame)."""
    return {k: float(((pred[:, sl] - label[:, sl]) ** 2).mean()) for k, sl in GROUPS.items()}


def train(X, Y, steps=3000, batch=4096, lr=1e-3, seed=0, log=print):
    net = InitMLP(seed=seed)
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    first = None
    for s in range(steps):
        idx = torch.randint(0, n, (batch,), generator=g).to(X.device)
        step_lr = lr * 0.5 * (1 + math.cos(math.pi * s / steps))
        loss = net.train_step(X[idx].contiguous(), Y[idx].contiguous(), lr=step_lr)
        first = loss if first is None else first
        if log and (s % 500 == 0 or s == steps - 1):
            log(f"  train step {s}: mse {loss:.4f}")
    return net, first, loss


def evaluate(net, seeds, iters=100, log=print, **case_kw):
    rows = []
    for s in seeds:
        c = Case(s, **case_kw)
        res = {"seed": s}
        for name, model in (("heuristic", None), ("learned", net)):
            P, fb, _ = c.initial_params(model)
            bm = c.mapper(P)
            l0 = final_loss(bm)
            lf, hist = run(bm, iters, record=True)
            res[name] = {"loss_init": l0, "loss_final": lf, "psnr_final": psnr_level0(bm), "fallback": fb,
                         "hist": hist}
        # iterations the learned start needs to reach the heuristic's final loss
        target = res["heuristic"]["loss_final"]
        h = res["learned"]["hist"]
        hit = np.nonzero(h <= target)[0]
        res["learned_iters_to_heuristic_final"] = int(hit[0]) if hit.size else None
        for name in ("heuristic", "learned"):
            res[name].pop("hist")
        if log:
            log(json.dumps(res))
        rows.append(res)
    hf = np.array([r["heuristic"]["loss_final"] for r in rows])
    lf = np.array([r["learned"]["loss_final"] for r in rows])
    hp = np.array([r["heuristic"]["psnr_final"] for r in rows])
    lp = np.array([r["learned"]["psnr_final"] for r in rows])
    return {"scenes": len(rows), "heuristic_loss_mean": hf.mean(), "heuristic_loss_std": hf.std(),
            "learned_loss_mean": lf.mean(), "learned_loss_std": lf.std(),
            "loss_gain_mean": (hf - lf).mean(), "loss_gain_std": (hf - lf).std(),
            "heuristic_psnr_mean": hp.mean(), "learned_psnr_mean": lp.mean(),
            "iters_to_heuristic_final": [r["learned_iters_to_heuristic_final"] for r in rows],
            "fallback": float(np.mean([r["learned"]["fallback"] for r in rows])), "rows": rows}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="small scenes, few seeds (a minute)")
    ap.add_argument("--train-seeds", type=int, default=20)
    ap.add_argument("--eval-seeds", type=int, default=5)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    kw = {}
    if a.quick:
        kw = dict(n=200_000, n_kf=4, per_kf=1024, kf_stride=1, min_weight=1.0)
        a.train_seeds, a.eval_seeds, a.steps = 6, 3, 1500
    t0 = time.time()
    X, Y, H = generate(range(a.train_seeds), a.iters, **kw)
    print(f"{X.shape[0]} pairs in {time.time() - t0:.1f}s", flush=True)
    # hold out every tenth pair to compare predictions with the heuristic in parameter space
    val = torch.arange(X.shape[0], device=X.device) % 10 == 0
    net, first, last = train(X[~val].contiguous(), Y[~val].contiguous(), a.steps)
    print(f"training mse {first:.4f} -> {last:.4f}", flush=True)
    pred = net.forward(X[val].contiguous())[:, :N_TARGET]
    perr = {"learned": param_errors(pred, Y[val]), "heuristic": param_errors(H[val], Y[val])}
    print("validation parameter mse " + json.dumps(perr), flush=True)
    res = evaluate(net, range(1000, 1000 + a.eval_seeds), a.iters, **kw)
    res["pairs"] = int(X.shape[0])
    res["validation_param_mse"] = perr
    res["train_mse"] = [first, last]
    summary = {k: v for k, v in res.items() if k != "rows"}
    print(json.dumps(summary, default=float), flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(res, fh, default=float, indent=1)


if __name__ == "__main__":
    main()
