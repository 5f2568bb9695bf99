"""Reports of the two extensions that change the method's numbers.

  python -m paper_2409_10383_amd.experiments precision [--steps 100]
      512 x 32^3 Brill-Lindquist + perturbations (dx = 0.125, 6th order):
      FP32 storage vs FP64 after n RK4 steps, per-field relative L2 / Linf
      errors and the Hamiltonian-constraint L2 (full and excised r >= 2).
  python -m paper_2409_10383_amd.experiments learned
      4096 x 16^3 two-puncture pack: train the indicator on h-vs-2h labels of
      varied puncture setups and report flag agreement against dchi-max.
  python -m paper_2409_10383_amd.experiments adaptive [--budget 64 --steps 16]
      the same training, then the closed loop: the `budget` blocks of the
      4096 x 16^3 pack of an unseen equal-mass setup that the learned
      indicator ranks highest, or that dchi-max ranks highest, are flagged;
      z4c_regrid_plan turns the flags into a refined mesh on which the
      puncture data are set (prolongating chi through a puncture overshoots
      below zero, so initial refinement re-evaluates the data, as mesh
      generation does); each mesh and the unrefined one are evolved and
      their constraint norms reported.
  python -m paper_2409_10383_amd.experiments blocksize [--steps 10]
      the linear wave of Sec. 4.1 on 256^3 zones split into MeshBlocks of
      16^3, 32^3, 64^3 (Table 1's size) and 128^3: zone-cycles per second of
      each, FP64, 6th order, autotuned launch (Sec. 5 reports the gain of
      larger MeshBlocks).

Each prints one JSON object.  All arithmetic runs in libz4c.
"""
import argparse
import json
import sys

import numpy as np


def precision(steps: int):
    import torch
    import paper_2409_10383_amd as z4c
    import z4c_inputs as zi
    mesh, p, data, dt, _ = zi.workload("bl512x32")
    print("precision: data ready", file=sys.stderr, flush=True)
    res = {}
    states = {}
    for prec, name in ((z4c.FP64, "fp64"), (z4c.FP32_MIXED, "fp32")):
        pk = z4c.Pack(mesh, p, prec)
        pk.upload(z4c.REG_U, data)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        pk.rk4_step(dt, steps)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        _, nf = pk.constraints(per_zone=False)
        _, ne = pk.constraints(per_zone=False, exclude=[(0.0, 0.0, 0.0)], r_exc=2.0)
        res[name] = {"zcps": pk.zones * steps / (ms * 1e-3), "H_L2": nf[0], "H_L2_excised": ne[0],
                     "M_L2": nf[2]}
        states[name] = pk.download(z4c.REG_U)
        print(f"precision: {name} run done", file=sys.stderr, flush=True)
        del pk
        torch.cuda.empty_cache()
    # a-priori bound of the FP32-storage error per field after n steps:
    #   storage rounding  n u32 max|f|
    # + derivative rounding  n dt K u32 (max|rhs_f| + S W2 / h^2)
    # (u32 = 2^-24; S = the largest |value| of the O(1) fields; W2 = sum of
    # |w| of the second-derivative stencil; K = 64 terms per right-hand side;
    # the FP64 accumulation is negligible), with max|f| and max|rhs_f| from
    # the FP64 run's initial state
    u32 = 2.0 ** -24
    pk = z4c.Pack(mesh, p, z4c.FP64)
    pk.upload(z4c.REG_U, data)
    pk.fill_ghosts()
    rhs0 = pk.split_interior(pk.rhs())
    del pk
    torch.cuda.empty_cache()
    S = max(float(np.abs(d[[0, 1, 4, 6, 18]]).max()) for d in data)
    w2 = float(np.sum(np.abs(z4c.stencil_weights(p["fd_order"])[1][1:]))) * 2 + \
        abs(float(z4c.stencil_weights(p["fd_order"])[1][0]))
    h = mesh.dx0
    err = {}
    for f in range(22):
        num2 = den2 = numi = deni = 0.0
        for a, b in zip(states["fp32"], states["fp64"]):
            d = a[f] - b[f]
            num2 += float(np.sum(d * d))
            den2 += float(np.sum(b[f] * b[f]))
            numi = max(numi, float(np.abs(d).max()))
            deni = max(deni, float(np.abs(b[f]).max()))
        fmax = max(float(np.abs(b[f]).max()) for b in data)
        rmax = max(float(np.abs(r[f]).max()) for r in rhs0)
        bound = steps * u32 * fmax + steps * dt * 64.0 * u32 * (rmax + S * w2 / h ** 2)
        err[zi.FIELDS[f]] = {"rel_L2": (num2 / max(den2, 1e-300)) ** 0.5,
                             "rel_Linf": numi / max(deni, 1e-300),
                             "Linf": numi, "apriori_bound": bound, "Linf_over_bound": numi / bound}
    out = {"workload": "bl512x32", "steps": steps, "dt": dt, "runs": res, "errors": err,
           "H_L2_ratio": res["fp32"]["H_L2"] / res["fp64"]["H_L2"],
           "H_L2_excised_ratio": res["fp32"]["H_L2_excised"] / res["fp64"]["H_L2_excised"]}
    print(json.dumps(out))


def _train(nvariants: int, epochs: int):
    """The indicator trained on h-vs-2h labels of `nvariants` random
    two-puncture setups on the 4096 x 16^3 pack; returns (net, snapshot,
    test setups, training samples, final MSE)."""
    import torch
    import paper_2409_10383_amd as z4c
    import z4c_inputs as zi
    p = zi.params_default(6)
    rng = np.random.default_rng(7)

    mesh = zi.uniform_mesh((16, 16, 16), 16, 4, (-16.0,) * 3, (16.0,) * 3, zi.BC_OUTFLOW)

    def snapshot(m1, m2, xp, yp, steps):
        """Two BL punctures (masses m1, m2) at (xp, yp, 0) and (-xp, -yp, 0);
        features and labels at the listed RK4 step counts."""
        print(f"snapshot m=({m1:.2f},{m2:.2f}) x=({xp:.2f},{yp:.2f}) steps={steps}", file=sys.stderr,
              flush=True)
        data = zi.brill_lindquist(mesh, [(m1, (xp, yp, 0.0)), (m2, (-xp, -yp, 0.0))])
        m2h = zi.coarse_2h_mesh(mesh)
        ph, p2 = z4c.Pack(mesh, p), z4c.Pack(m2h, p)
        ph.upload(z4c.REG_U, data)
        F, Y, D, flags = [], [], [], []
        done = 0
        for s in steps:
            ph.rk4_step(0.25 * mesh.dx0, s - done)
            done = s
            z4c.inject_2h(ph, p2)
            ph.fill_ghosts()
            p2.fill_ghosts()
            Y.append(z4c.labels(ph, ph.rhs(), p2, p2.rhs()))
            dev = torch.empty(mesh.nb * 16, dtype=torch.float64, device="cuda")
            F.append(z4c.features(ph, device_out=dev))
            D.append(dev.view(mesh.nb, 16))
        return F, Y, D

    def setup():
        return (rng.uniform(0.3, 0.7), rng.uniform(0.3, 0.7), rng.uniform(3.0, 7.0),
                rng.uniform(-1.0, 1.0))
    train = [setup() for _ in range(nvariants)]
    test = [(0.5, 0.5, 5.0, 0.0), setup()]
    Ftr, Ytr, Dtr = [], [], []
    for v in train:
        F, Y, D = snapshot(*v, steps=(0, 8))
        Ftr += F; Ytr += Y; Dtr += D
    net = z4c.Mlp(zi.mlp_init(1))
    Dall = torch.cat(Dtr)
    net.fit_stats(Dall)
    X = net.normalize(Dall)
    T = torch.tensor(np.concatenate(Ytr).astype(np.float32), device="cuda")
    print(f"training on {T.numel()} blocks", file=sys.stderr, flush=True)
    loss = net.train(X, T, epochs=epochs, lr=3e-3, batch=4096)
    print(f"final training MSE {loss:.4f}", file=sys.stderr, flush=True)
    return net, snapshot, test, int(T.numel()), loss


def learned(nvariants: int = 6, epochs: int = 40):
    net, snapshot, test, ntrain, loss = _train(nvariants, epochs)
    rows = []
    for v in test:
        F, Y, D = snapshot(*v, steps=(0,))
        pred = net.forward(net.normalize(D[0])).cpu().numpy()
        y, f = Y[0], F[0]
        for K in (64, 256):
            truth = set(np.argsort(-y)[:K])
            rows.append({"setup": list(map(float, v)), "K": K,
                         "learned_precision": len(truth & set(np.argsort(-pred)[:K])) / K,
                         "dchi_max_precision": len(truth & set(np.argsort(-f[:, 0])[:K])) / K})
    print(json.dumps({"workload": "bbh4096x16", "train_samples": ntrain,
                      "final_mse": loss, "test": rows}))


def adaptive(budget: int = 64, steps: int = 16, nvariants: int = 6, epochs: int = 40):
    import torch
    import paper_2409_10383_amd as z4c
    import z4c_inputs as zi
    net, _, test, ntrain, loss = _train(nvariants, epochs)
    p = zi.params_default(6)
    mesh = zi.uniform_mesh((16, 16, 16), 16, 4, (-16.0,) * 3, (16.0,) * 3, zi.BC_OUTFLOW)
    m1, m2, xp, yp = test[0]
    punct = [(xp, yp, 0.0), (-xp, -yp, 0.0)]
    data = zi.brill_lindquist(mesh, [(m1, punct[0]), (m2, punct[1])])
    base = z4c.Pack(mesh, p)
    base.upload(z4c.REG_U, data)
    base.fill_ghosts()
    masses = [(m1, punct[0]), (m2, punct[1])]
    dev = torch.empty(mesh.nb * 16, dtype=torch.float64, device="cuda")
    feat = z4c.features(base, device_out=dev)
    pred = net.forward(net.normalize(dev.view(mesh.nb, 16))).cpu().numpy()
    ranks = {"learned": np.argsort(-pred)[:budget], "dchi_max": np.argsort(-feat[:, 0])[:budget]}
    runs = {}
    for name in ("none", "learned", "dchi_max"):
        if name == "none":
            pk = z4c.Pack(mesh, p)
            pk.upload(z4c.REG_U, data)
        else:
            flags = np.zeros(mesh.nb, np.int8)
            flags[ranks[name]] = 1
            new = base.regrid_plan(flags, level_max=1)
            pk = z4c.Pack(new, p)
            pk.upload(z4c.REG_U, zi.brill_lindquist(new, masses))
        # every mesh evolves to t = steps * 0.25 dx of the unrefined mesh
        dt = 0.25 * pk.mesh.dx_min()
        nst = int(round(steps * 0.25 * mesh.dx_min() / dt))
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        pk.rk4_step(dt, nst)
        t1.record()
        torch.cuda.synchronize()
        _, nf = pk.constraints(per_zone=False)
        _, ne = pk.constraints(per_zone=False, exclude=punct, r_exc=1.0)
        runs[name] = {"blocks": int(pk.mesh.nb), "zones": int(pk.zones), "dt": dt, "steps": nst,
                      "t_end": dt * nst, "ms": t0.elapsed_time(t1),
                      "H_L2": float(nf[0]), "H_Linf": float(nf[1]), "M_L2": float(nf[2]),
                      "H_L2_excised_r1": float(ne[0])}
        print(f"{name}: {runs[name]}", file=sys.stderr, flush=True)
        del pk
        torch.cuda.empty_cache()
    overlap = len(set(ranks["learned"].tolist()) & set(ranks["dchi_max"].tolist()))
    print(json.dumps({"workload": "bbh4096x16 adaptive", "setup": list(map(float, test[0])),
                      "budget_blocks": budget, "train_samples": ntrain, "final_mse": loss,
                      "flag_overlap": overlap, "runs": runs}))


def blocksize(steps: int = 10):
    import torch
    import paper_2409_10383_amd as z4c
    import z4c_inputs as zi
    p = zi.params_default(6)
    rows = []
    for n in (16, 32, 64, 128):
        mesh, data = zi.linear_wave_pack(256 // n, n)
        pk = z4c.Pack(mesh, p)
        pk.upload(z4c.REG_U, data)
        del data
        chosen, _ = pk.autotune(reps=3)
        dt = 0.25 * mesh.dx0
        pk.rk4_step(dt, 2)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        pk.rk4_step(dt, steps)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        pk.profile(True)
        pk.profile_read(reset=True)
        pk.rk4_step(dt, 1)
        st_ms, st_n, fill_ms, fill_n, _, _ = pk.profile_read(reset=True)
        row = {"block": n, "blocks": int(mesh.nb), "zones": int(pk.zones),
               "zcps": pk.zones * steps / (ms * 1e-3), "ms_per_step": ms / steps,
               "stage_ms": st_ms / st_n, "fill_ms": fill_ms / max(fill_n, 1),
               "tile": "x".join(str(v) for v in z4c.TILE_SHAPES[chosen // 2]),
               "persistent": bool(chosen % 2)}
        print(row, file=sys.stderr, flush=True)
        rows.append(row)
        del pk
        torch.cuda.empty_cache()
    print(json.dumps({"workload": "linear wave, 256^3 zones, periodic unit cube", "fd_order": 6,
                      "precision": "fp64", "steps": steps, "rows": rows}))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["precision", "learned", "adaptive", "blocksize"])
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--budget", type=int, default=64)
    a = ap.parse_args(argv)
    if a.what == "precision":
        precision(a.steps or 100)
    elif a.what == "learned":
        learned()
    elif a.what == "blocksize":
        blocksize(a.steps or 10)
    else:
        adaptive(a.budget, a.steps or 16)


if __name__ == "__main__":
    sys.exit(main())
