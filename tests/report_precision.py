"""Per-triplet error of both GPU precisions against the full FP64 oracle
at the headline workload (256^3, 30 bins, 3035 triplets).

Not collected by pytest (runs ~1 min of oracle work):
    python tests/report_precision.py [out.json]
Prints a summary table and writes the per-triplet errors as JSON.
"""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import paper_2404_07249_amd as pb3  # noqa: E402
from synthetic import field_for  # noqa: E402


def main():
    import torch

    out = sys.argv[1] if len(sys.argv) > 1 else None
    d, cfg = field_for("c3")
    plan = pb3.Plan(cfg["n"], cfg["box"], cfg["edges"])
    x = torch.from_numpy(d).cuda()
    gpu = {}
    for prec in ("fp32", "mixed"):
        pk, bk = plan.polyspectra(x, prec)
        torch.cuda.synchronize()
        gpu[prec] = (pk.cpu().numpy(), bk.cpu().numpy())
    print("[report] GPU done; running the FP64 oracle", flush=True)
    t0 = time.time()
    _, cnt = plan.norm()
    res = oracle.bispectrum(d.astype(np.float64), cfg["box"], cfg["edges"], plan.triplets.astype(np.int64),
                            cnt.astype(np.int64))
    print(f"[report] oracle {time.time() - t0:.1f} s", flush=True)
    rep = {"workload": "256^3, L=2000, 30 bins, 3035 triplets, seed 2", "triplets": res.triplets.tolist()}
    for prec, (pk, bk) in gpu.items():
        db = np.abs(bk - res.bk)
        rel = db / np.abs(res.bk)
        byA = db / res.absnorm
        gate = db <= 1e-5 * np.abs(res.bk) + 1e-6 * res.absnorm
        prel = np.abs(pk - res.pk) / np.abs(res.pk)
        summary = {
            "P_rel_max": float(prel.max()),
            "B_absA_max": float(byA.max()),
            "B_rel_median": float(np.median(rel)),
            "B_rel_p99": float(np.percentile(rel, 99)),
            "B_rel_max": float(rel.max()),
            "frac_rel_le_1e-5": float(np.mean(rel <= 1e-5)),
            "gate_pass": int(gate.sum()),
            "n": int(len(bk)),
        }
        rep[prec] = {"summary": summary, "dB_over_A": byA.tolist(), "rel": rel.tolist()}
        print(prec, json.dumps(summary), flush=True)
    print("kappa (A/|B|): median %.3g p99 %.3g max %.3g" % (np.median(res.kappa), np.percentile(res.kappa, 99),
                                                            res.kappa.max()))
    if out:
        with open(out, "w") as f:
            json.dump(rep, f)


if __name__ == "__main__":
    main()
