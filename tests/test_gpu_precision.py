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
from bars import GRAD_TOL, KL_TOL, P_TOL, ROW_TOL, Z_TOL, kl_close, rel_l2, row_error_ratio, sample_rows
from paper_2310_11186_amd import synth, tsgne

pytestmark = pytest.mark.gpu

OUT = os.environ.get("TSGNE_REPORT_DIR", "")


def write_report(key, entry):
    """Adds one entry to precision_report.json under TSGNE_REPORT_DIR (if set)."""
    if not (OUT and os.path.isdir(OUT)):
        return
    path = os.path.join(OUT, "precision_report.json")
    report = json.load(open(path)) if os.path.exists(path) else {}
    report[key] = entry
    with open(path, "w") as fh:
        json.dump(report, fh, indent=1)


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
            okl = oracle.kl(rp, col, oP, Yg.cpu().numpy().astype(np.float64))
            res["kl_abs"] = abs(tsgne.tsgne_kl(g, Yg) - okl)
            res["kl_rel"] = res["kl_abs"] / max(1.0, abs(okl))
            entry[mode_name] = res
        report[name] = entry
        g.close()
        write_report(name, entry)
        sp, fp = entry["split"], entry["fp32"]
        assert entry["P_rel_l2"] <= P_TOL
        for sname in states:
            assert sp[sname]["grad_rel_l2"] <= GRAD_TOL and sp[sname]["Z_rel"] <= Z_TOL
            assert fp[sname]["grad_rel_l2"] <= 1e-3 and fp[sname]["Z_rel"] <= 1e-4
        assert sp["traj30_rel_l2"] <= 3 * sp["traj30_fp32_state_oracle_drift"] + 1e-4
        assert sp["kl_rel"] <= KL_TOL
    print(json.dumps(report, indent=1))




# States of the 1000-iteration schedule at which the c3 checks compare: the
# start, the first steps, the end of early exaggeration (t = 250) and its
# eve, half way, and the end.
C3_STATES = (0, 1, 10, 125, 250, 500, 1000)
C3_ITERS, C3_TEE = 1000, 250
# Bars on the final KL of the 1000-iteration snowball layouts relative to the
# oracle's.  The layout is a chaotic function of rounding in the early phase:
# the FP64 oracle itself, started from Y0 perturbed by 1e-7 relative (five
# seeds), ends at -0.25 %, +0.22 %, -0.32 %, +0.07 % and +0.18 % of its
# unperturbed run's final KL (4.7682); the bars are about three times the
# widest of those (measured on the GPU: split -0.02 %, all-FP32 +0.30 %).
C3_KL_BAR_SPLIT = 0.01
C3_KL_BAR_FP32 = 0.01


def shadow_step(g, gpu, p, t, s, orp, ocol, oP, eta, early_exaggeration=12.0):
    """One GPU step from the oracle state s = (Y, U, gains) rounded to FP32,
    against one oracle step from the same state: (gradient rel L2, worst
    per-row ratio, update rel L2 outside gain flips, flips)."""
    import torch
    Y, U, G = (f32(a) for a in s)
    alpha, mom = (early_exaggeration, 0.5) if t < C3_TEE else (1.0, 0.8)
    og, oZ = oracle.gradient(orp, ocol, oP, Y, alpha)
    oY1, oU1, oG1 = oracle.update(Y, U, G, og, mom, eta)
    dY, dU, dG = (torch.from_numpy(a.astype(np.float32)).to(gpu) for a in (Y, U, G))
    gg = torch.empty_like(dY)
    tsgne.tsgne_step(g, dY, dU, dG, t, p, grad_out=gg)
    gg = gg.cpu().numpy().astype(np.float64)
    gU, gG = dU.cpu().numpy().astype(np.float64), dG.cpu().numpy().astype(np.float64)
    same = np.abs(gG - oG1) <= 1e-6 * np.abs(oG1)   # the gain branch taken alike
    return (rel_l2(gg, og), row_error_ratio(gg, og, Y, oZ)[0], rel_l2(gU[same], oU1[same]), int((~same).sum()))


def test_precision_c3_subsample(gpu):
    """The 300K-node graph's precision check on a 20,000-node BFS snowball
    sample over the whole schedule: 1000 iterations with early exaggeration
    for the first 250, the learning rate n / 48, in the split mode and in
    all-FP32, against the FP64 oracle.

    At each state of C3_STATES on the oracle's trajectory (rounded to FP32)
    one GPU step is checked against one oracle step (gradient, per-row bound,
    update vector, Z); the final layouts are compared through KL, whose
    spread under a 1e-7 perturbation of Y0 sets that bar (the layout itself
    is a chaotic function of the rounding, reported only)."""
    import torch
    sub = synth.snowball_sample(synth.make("dcsbm300k"), 20_000, seed=1)
    rp, col = tsgne.tsgne_csr_from_edges(sub.n, sub.edges)
    g = tsgne.tsgne_build_P(torch.from_numpy(rp).to(gpu), torch.from_numpy(col).to(gpu),
                            torch.from_numpy(sub.X).to(gpu), 30.0)
    oP, _ = oracle.build_P(rp, col, sub.X, 30.0)
    eta = max(sub.n / 48.0, 50.0)
    entry = {"nodes": sub.n, "edges": int(sub.edges.shape[0]), "iterations": C3_ITERS,
             "exaggeration_iters": C3_TEE, "eta": eta, "P_rel_l2": rel_l2(g.export()["P"], oP)}
    # the oracle's trajectory, kept at the checked states
    s = (sub.Y0.astype(np.float64), np.zeros((sub.n, 2)), np.ones((sub.n, 2)))
    ostates = {0: s}
    t = 0
    for t_next in C3_STATES[1:]:
        Y, U, G, _ = oracle.run(rp, col, oP, *s, t0=t, n_steps=t_next - t, exaggeration_iters=C3_TEE, eta=eta)
        s, t = (Y, U, G), t_next
        ostates[t] = s
        write_report("dcsbm300k_snowball20k_progress", {"oracle_t": t})
    oY = ostates[C3_ITERS][0]
    o_kl = oracle.kl(rp, col, oP, oY)
    entry["oracle_kl"] = o_kl
    for name, mode in (("split", tsgne.TSGNE_PREC_SPLIT), ("fp32", tsgne.TSGNE_PREC_FP32)):
        p = tsgne.tsgne_params_default(precision=mode, exaggeration_iters=C3_TEE, learning_rate=eta)
        per_state = {}
        for t in C3_STATES:
            Yt = f32(ostates[t][0])
            alpha = 12.0 if t < C3_TEE else 1.0
            og, oZ = oracle.gradient(rp, col, oP, Yt, alpha)
            grad, Z = tsgne.tsgne_gradient(g, torch.from_numpy(Yt.astype(np.float32)).to(gpu), alpha, p)
            gg = grad.cpu().numpy()
            st = {"grad_rel_l2": rel_l2(gg, og), "grad_row_ratio": row_error_ratio(gg, og, Yt, oZ)[0],
                  "Z_rel": abs(Z.item() / oZ - 1.0)}
            if t < C3_ITERS:
                st["step_grad_rel_l2"], st["step_row_ratio"], st["step_update_rel_l2"], st["gain_flips"] = \
                    shadow_step(g, gpu, p, t, ostates[t], rp, col, oP, eta)
            per_state[str(t)] = st
        Yg = torch.from_numpy(sub.Y0).to(gpu)
        tsgne.tsgne_run(g, Yg, C3_ITERS, p)
        kl = tsgne.tsgne_kl(g, Yg)
        entry[name] = {"states": per_state, "kl": kl, "kl_rel_to_oracle": kl / o_kl - 1.0,
                       "layout_rel_l2": rel_l2(Yg.cpu().numpy(), oY)}
        write_report("dcsbm300k_snowball20k", entry)
    g.close()
    print(json.dumps(entry, indent=1))
    sp, fp = entry["split"], entry["fp32"]
    assert entry["P_rel_l2"] <= P_TOL
    for t, st in sp["states"].items():
        assert st["grad_rel_l2"] <= GRAD_TOL and st["grad_row_ratio"] <= ROW_TOL, (t, st)
        assert st["Z_rel"] <= Z_TOL, (t, st)
        if "step_grad_rel_l2" in st:
            assert st["step_grad_rel_l2"] <= GRAD_TOL and st["step_row_ratio"] <= ROW_TOL, (t, st)
            assert st["step_update_rel_l2"] <= GRAD_TOL, (t, st)
            assert st["gain_flips"] <= 1e-3 * 2 * sub.n, (t, st)
    for t, st in fp["states"].items():
        assert st["grad_rel_l2"] <= 1e-3 and st["Z_rel"] <= 1e-4, (t, st)
    assert abs(sp["kl_rel_to_oracle"]) <= C3_KL_BAR_SPLIT
    assert abs(fp["kl_rel_to_oracle"]) <= C3_KL_BAR_FP32


def test_c3_trajectory_states_full_graph(gpu):
    """The 300K-node graph itself along the GPU's own 1000-iteration layout
    (default parameters: early exaggeration 12 for 250 iterations, learning
    rate n / 48, automatic tile, precision split): at every state of
    C3_STATES the gradient of sampled rows (512 seeded random rows, the first
    and last rows and the first row of the last block of every tile length),
    Z over all 9e10 ordered pairs and KL are checked against the FP64 oracle
    at the same FP32 state."""
    import torch
    gi = synth.make("dcsbm300k")
    rp, col = tsgne.tsgne_csr_from_edges(gi.n, gi.edges)
    g = tsgne.tsgne_build_P(torch.from_numpy(rp).to(gpu), torch.from_numpy(col).to(gpu),
                            torch.from_numpy(gi.X).to(gpu), 30.0)
    oP, _ = oracle.build_P(rp, col, gi.X, 30.0)
    p = tsgne.tsgne_params_default(exaggeration_iters=C3_TEE)
    rows = sample_rows(gi.n, 512, 23)
    Y = torch.from_numpy(gi.Y0).to(gpu)
    U, G = torch.zeros_like(Y), torch.ones_like(Y)
    snaps = {}
    t = 0
    for t_next in C3_STATES:
        while t < t_next:
            tsgne.tsgne_step(g, Y, U, G, t, p)
            t += 1
        snaps[t] = Y.cpu().numpy()
    entry = {}
    for t in C3_STATES:
        Yt = snaps[t]
        alpha = 12.0 if t < C3_TEE else 1.0
        grad, Z = tsgne.tsgne_gradient(g, torch.from_numpy(Yt).to(gpu), alpha, p)
        kl = tsgne.tsgne_kl(g, torch.from_numpy(Yt).to(gpu))
        og, oZ = oracle.gradient_rows(rp, col, oP, Yt.astype(np.float64), rows, alpha)
        gg = grad.cpu().numpy()[rows]
        entry[str(t)] = {"grad_rel_l2": rel_l2(gg, og), "grad_row_ratio": row_error_ratio(gg, og, Yt, oZ, rows)[0],
                         "Z_rel": abs(Z.item() / oZ - 1.0),
                         "kl": kl, "kl_oracle": oracle.kl_given_Z(rp, col, oP, Yt.astype(np.float64), oZ)}
        write_report("dcsbm300k_trajectory_states", entry)
    g.close()
    print(json.dumps(entry, indent=1))
    for t, st in entry.items():
        assert st["grad_rel_l2"] <= GRAD_TOL and st["grad_row_ratio"] <= ROW_TOL, (t, st)
        assert st["Z_rel"] <= Z_TOL and kl_close(st["kl"], st["kl_oracle"]), (t, st)
