"""The paper's 1-D mixture simulation on the GPU (Sec. 3.2; App. A.3): fit GMM, DoG, LoG and GEF mixtures of
N components to the six 1-D signals, 20 seeded runs per configuration, and print the mean final MSE per model
and N for each signal with the number of NaN runs.

    python -m paper_2402_10128_amd.mixture_sim [--epochs 1000] [--runs 20] [--weights positive|free|both]

Every fit runs in one launch of the library's batched kernel (ges_mix_fit); this module only builds the
problem table from the seeded workload and formats the result.
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import torch

from . import ges as G
from . import synth

MODELS = ("gmm", "dog", "log", "gef")


def run(epochs: int = 1000, runs: int = 20, weights=("positive", "free"), seed: int = 0, lr: float = 0.01,
        device: str = "cuda:0") -> dict:
    W = synth.mixture_workload(seed=seed, runs=runs, weights=weights)
    dev = torch.device(device)
    probs = torch.from_numpy(W["problems"]).to(dev)
    params = torch.from_numpy(W["params"]).to(dev)
    loss = G.ges_mix_fit(probs, torch.from_numpy(W["targets"]).to(dev), W["x0"], W["dx"], params, epochs, lr)
    loss = loss.cpu().numpy()
    pr = W["problems"]
    table = {}
    for s_i, sig in enumerate(synth.MIX_SIGNALS):
        for mode in weights:
            pos = 1 if mode == "positive" else 0
            rows = {}
            for k, name in enumerate(MODELS):
                cells = {}
                for n in synth.MIX_NS:
                    sel = (pr[:, 0] == k) & (pr[:, 1] == n) & (pr[:, 3] == s_i) & (pr[:, 2] == pos)
                    v = loss[sel]
                    fin = np.isfinite(v)
                    cells[n] = (float(v[fin].mean()) if fin.any() else float("nan"), int((~fin).sum()))
                rows[name] = cells
            table[(sig, mode)] = rows
    return {"table": table, "epochs": epochs, "runs": runs, "problems": int(len(pr))}


def format_table(res: dict) -> str:
    out = []
    for (sig, mode), rows in res["table"].items():
        out.append(f"signal {sig}, {mode} weights: mean final MSE over {res['runs']} runs (NaN runs in brackets)")
        out.append("  model " + "".join(f"{'N=' + str(n):>14s}" for n in synth.MIX_NS))
        for name, cells in rows.items():
            line = f"  {name:5s} "
            for n in synth.MIX_NS:
                mse, nan = cells[n]
                line += f"{mse:>10.2e}" + (f"[{nan:2d}]" if nan else "    ")
            out.append(line)
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--epochs", type=int, default=1000)
    ap.add_argument("--runs", type=int, default=20)
    ap.add_argument("--weights", choices=["positive", "free", "both"], default="both")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--json", action="store_true", help="print the table as JSON")
    args = ap.parse_args()
    weights = ("positive", "free") if args.weights == "both" else (args.weights,)
    res = run(args.epochs, args.runs, weights, args.seed)
    if args.json:
        print(json.dumps({f"{s}/{m}": {k: {str(n): c for n, c in v.items()} for k, v in rows.items()}
                          for (s, m), rows in res["table"].items()}))
    else:
        print(format_table(res))


if __name__ == "__main__":
    main()
