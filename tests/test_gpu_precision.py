"""Error of each result against FP64 for the two precision modes.

TSGNE_PREC_SPLIT: FP32 pair arithmetic, FP64 for Z, the cross-tile force sums,
the attraction sums and KL.  TSGNE_PREC_FP32: everything in FP32.  P is
computed in FP64 and stored in FP32 in both modes.  The measured table is
written to precision_report.json in the folder named by the environment
variable TSGNE_REPORT_DIR, when it is set and exists; the assertions are the
bars for the split mode and loose sanity bounds for FP32.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2310_11186_amd import synth, tsgne

pytestmark = pytest.mark.gpu

OUT = os.environ.get("TSGNE_REPORT_DIR", "")


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def f32(a):
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def fp32_state_drift(rp, col, oP, Y0, steps, oY):
    """Drift of the oracle itself when its P and state are rounded to FP32
    between steps: the floor any FP32-state implementation can reach."""
    P32 = f32(oP)
    Y, U, G = f32(Y0), np.zeros_like(Y0, np.float64), np.ones_like(Y0, np.float64)
    for t in range(steps):
        Y, U, G, _ = oracle.run(rp, col, P32, Y, U, G, t0=t, n_steps=1, exaggeration_iters=125, eta=50.0)
        Y, U, G = f32(Y), f32(U), f32(G)
    return rel_l2(Y, oY)


def test_precision_split_vs_fp32(gpu):
    import torch
    report = {}
    cases = {"sbm2k": synth.make("sbm2k"), "dcsbm3001": synth.small_dcsbm(3001, 9003, 2.4, 15, 8, 5)}
    for name, gi in cases.items():
        rp, col = tsgne.tsgne_csr_from_edges(gi.n, gi.edges)
        g = tsgne.tsgne_build_P(torch.from_numpy(rp).to(gpu), torch.from_numpy(col).to(gpu),
                                torch.from_numpy(gi.X).to(gpu), 30.0)
        oP, _ = oracle.build_P(rp, col, gi.X, 30.0)
        P32 = g.export()["P"]
        entry = {"P_rel_l2": rel_l2(P32, oP)}
        rng = np.random.default_rng(1)
        states = {"y0": gi.Y0, "spread1": rng.standard_normal((gi.n, 2)).astype(np.float32),
                  "spread30": (30 * rng.standard_normal((gi.n, 2))).astype(np.float32)}
        for mode_name, mode in (("split", tsgne.TSGNE_PREC_SPLIT), ("fp32", tsgne.TSGNE_PREC_FP32)):
            p = tsgne.tsgne_params_default(precision=mode, exaggeration_iters=125, learning_rate=50.0)
            res = {}
            for sname, Y in states.items():
                og, oZ = oracle.gradient(rp, col, oP, Y.astype(np.float64), 1.0)
                grad, Z = tsgne.tsgne_gradient(g, torch.from_numpy(Y).to(gpu), 1.0, p)
                res[sname] = {"grad_rel_l2": rel_l2(grad.cpu().numpy(), og), "Z_rel": abs(Z.item() / oZ - 1.0)}
            # 30 steps from Y0, beside the FP32-state oracle's own drift
            oY, _, _, _ = oracle.run(rp, col, oP, gi.Y0, n_steps=30, exaggeration_iters=125, eta=50.0)
            Yg = torch.from_numpy(gi.Y0).to(gpu)
            tsgne.tsgne_run(g, Yg, 30, p)
            res["traj30_rel_l2"] = rel_l2(Yg.cpu().numpy(), oY)
            res["traj30_fp32_state_oracle_drift"] = fp32_state_drift(rp, col, oP, gi.Y0, 30, oY)
            res["kl_abs"] = abs(tsgne.tsgne_kl(g, Yg) - oracle.kl(rp, col, oP, Yg.cpu().numpy().astype(np.float64)))
            entry[mode_name] = res
        report[name] = entry
        g.close()
        if OUT and os.path.isdir(OUT):
            with open(os.path.join(OUT, "precision_report.json"), "w") as f:
                json.dump(report, f, indent=1)
        sp, fp = entry["split"], entry["fp32"]
        assert entry["P_rel_l2"] <= 1e-6
        for sname in states:
            assert sp[sname]["grad_rel_l2"] <= 1e-5 and sp[sname]["Z_rel"] <= 1e-6
            assert fp[sname]["grad_rel_l2"] <= 1e-3 and fp[sname]["Z_rel"] <= 1e-4
        assert sp["traj30_rel_l2"] <= 3 * sp["traj30_fp32_state_oracle_drift"] + 1e-4
        assert sp["kl_abs"] <= 1e-6
    print(json.dumps(report, indent=1))


def test_precision_c3_subsample(gpu):
    """The 300K-node graph's precision check on a 20,000-node BFS snowball
    sample: 250 steps in the split mode and in all-FP32 against the FP64
    oracle (KL of the final layouts; gradient and Z at the oracle's final
    state, where the comparison is free of trajectory chaos)."""
    import torch
    sub = synth.snowball_sample(synth.make("dcsbm300k"), 20_000, seed=1)
    steps, t_ee = 250, 62
    rp, col = tsgne.tsgne_csr_from_edges(sub.n, sub.edges)
    g = tsgne.tsgne_build_P(torch.from_numpy(rp).to(gpu), torch.from_numpy(col).to(gpu),
                            torch.from_numpy(sub.X).to(gpu), 30.0)
    oP, _ = oracle.build_P(rp, col, sub.X, 30.0)
    eta = max(sub.n / 48.0, 50.0)
    oY, _, _, _ = oracle.run(rp, col, oP, sub.Y0, n_steps=steps, exaggeration_iters=t_ee, eta=eta)
    o_kl = oracle.kl(rp, col, oP, oY)
    og, oZ = oracle.gradient(rp, col, oP, oY, 1.0)
    entry = {"nodes": sub.n, "edges": int(sub.edges.shape[0]), "steps": steps, "oracle_kl": o_kl,
             "P_rel_l2": rel_l2(g.export()["P"], oP)}
    for name, mode in (("split", tsgne.TSGNE_PREC_SPLIT), ("fp32", tsgne.TSGNE_PREC_FP32)):
        p = tsgne.tsgne_params_default(precision=mode, exaggeration_iters=t_ee, learning_rate=eta)
        Yg = torch.from_numpy(sub.Y0).to(gpu)
        tsgne.tsgne_run(g, Yg, steps, p)
        kl = tsgne.tsgne_kl(g, Yg)
        grad, Z = tsgne.tsgne_gradient(g, torch.from_numpy(oY.astype(np.float32)).to(gpu), 1.0, p)
        og32, _ = oracle.gradient(rp, col, oP, f32(oY), 1.0)      # the oracle at the same FP32-rounded state
        entry[name] = {"kl": kl, "kl_rel_to_oracle": kl / o_kl - 1.0,
                       "grad_rel_l2_at_oracle_state": rel_l2(grad.cpu().numpy(), og32),
                       "Z_rel_at_oracle_state": abs(Z.item() / oZ - 1.0),
                       "traj_rel_l2": rel_l2(Yg.cpu().numpy(), oY)}
    g.close()
    if OUT and os.path.isdir(OUT):
        path = os.path.join(OUT, "precision_report.json")
        report = json.load(open(path)) if os.path.exists(path) else {}
        report["dcsbm300k_snowball20k"] = entry
        with open(path, "w") as fh:
            json.dump(report, fh, indent=1)
    print(json.dumps(entry, indent=1))
    sp, fp = entry["split"], entry["fp32"]
    assert entry["P_rel_l2"] <= 1e-6
    assert sp["grad_rel_l2_at_oracle_state"] <= 1e-5 and sp["Z_rel_at_oracle_state"] <= 1e-5
    # After 250 steps the layout is past the chaotic early phase: the FP64
    # oracle itself, started from Y0 perturbed by 1e-7 relative, ends with KL
    # between -0.9 % and +3.4 % of its unperturbed run (5 perturbed runs), so
    # the final KL is held to a bar above that spread, not to rounding error
    assert abs(sp["kl_rel_to_oracle"]) <= 0.05
    assert fp["grad_rel_l2_at_oracle_state"] <= 1e-3 and abs(fp["kl_rel_to_oracle"]) <= 0.08
