"""Write sampled snapshots of the FP64 oracle on the 2e7-dof sphere-band mesh (2000 steps).

The oracle cannot run inside a GPU test at this size (about an hour on 8 host cores), so
this script runs it once and stores, for every 100th step:

* the infinity norm of the whole displacement field (the normaliser of the relative error);
* the displacements of a fixed seeded sample of nodes and of the node where |u| is largest;
* the discrete energy H_{n+1/2} and the external work W_n of the run.

The GPU tests compare the library's trajectory with these values.  Only the oracle and the
seeded input generator are called; the mesh fingerprint lets a test refuse the file when a
regenerated mesh differs.

Usage: python tests/golden/make_oracle_snapshots.py [--steps 2000] [--every 100] [--out PATH]
"""

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N_SAMPLE = 512


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--out", default=os.path.join(HERE, "cfg4_oracle_snapshots.txt"))
    args = ap.parse_args()
    from meshgen import configs
    from oracle.solver import Oracle  # the writer only: read() below parses the file alone
    t0 = time.time()
    mesh = configs.cfg4(n_steps=args.steps)
    o = Oracle(mesh, workers=args.workers)
    dt = mesh.load["dt_factor"] * o.critical_dt()
    rng = np.random.default_rng([4, 2000])
    free_nodes = np.flatnonzero(~mesh.fixed.reshape(-1, 3).all(1))
    sample = np.sort(rng.choice(free_nodes, N_SAMPLE, replace=False))
    print(f"cfg4: {mesh.n_dof} dofs, {mesh.n_cells} cells, dt {dt:.6e}, set-up {time.time() - t0:.0f} s", flush=True)

    u, um1 = o.initial_state(dt)
    d = u - um1
    H_prev = 0.5 * (d @ (o.mdiag * d)) / dt ** 2 + 0.5 * (u @ o.internal_force(um1))
    H0, W = H_prev, 0.0
    rows = []
    t1 = time.time()
    for n in range(args.steps):
        unew, f = o.step(u, um1, n, dt)
        d = unew - u
        H = 0.5 * (d @ (o.mdiag * d)) / dt ** 2 + 0.5 * (unew @ f)
        W += 0.5 * ((unew - um1) @ (o.load_at(n * dt) * o.b))
        um1, u = u, unew
        k = n + 1
        if k % args.every == 0 or k == args.steps:
            a = np.abs(u)
            imax = int(np.argmax(a))
            rows.append(dict(step=k, norm=float(a.max()), imax=imax // 3, H=float(H), W=float(W),
                             u=u.reshape(-1, 3)[sample].copy(), umax=u.reshape(-1, 3)[imax // 3].copy()))
            el = time.time() - t1
            print(f"step {k}: |u|_inf {a.max():.6e}, H {H:.6e}, {el:.0f} s ({mesh.n_dof * k / el:.3e} dof-steps/s)",
                  flush=True)
    drift = max(abs(r["H"] - H0 - r["W"]) for r in rows) / max(abs(r["H"]) for r in rows)
    lines = [
        "# Sampled snapshots of the FP64 oracle (Alg. 1, eq. DnMdiag) on the sphere-band octree, levels 4/8",
        f"# written by tests/golden/make_oracle_snapshots.py in {time.time() - t0:.0f} s",
        f"mesh_fingerprint {mesh.fingerprint()}",
        f"n_dof {mesh.n_dof}",
        f"n_cells {mesh.n_cells}",
        f"dt {float(dt)!r}",
        f"steps {args.steps}",
        f"every {args.every}",
        f"H0 {float(H0)!r}",
        f"energy_drift_at_snapshots {float(drift)!r}",
        "sample_nodes " + " ".join(str(int(v)) for v in sample),
        "# per snapshot: step, |u|_inf over all dofs, node of the largest |u|, H_{n+1/2}, W_n,",
        "# the three displacements of that node, then of every sample node in order",
    ]
    for r in rows:
        vals = [repr(float(v)) for v in r["umax"]] + [repr(float(v)) for v in r["u"].ravel()]
        lines.append(f"snap {r['step']} {r['norm']!r} {r['imax']} {r['H']!r} {r['W']!r} " + " ".join(vals))
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {args.out}", flush=True)


def read(path):
    """Parse a snapshot file: dict with the header values, sample nodes and snapshot rows."""
    out = dict(snaps=[])
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        key, rest = line.split(" ", 1)
        rest = rest.split()
        if key == "snap":
            out["snaps"].append(dict(step=int(rest[0]), norm=float(rest[1]), imax=int(rest[2]), H=float(rest[3]),
                                     W=float(rest[4]), umax=np.array([float(v) for v in rest[5:8]]),
                                     u=np.array([float(v) for v in rest[8:]]).reshape(-1, 3)))
        elif key == "sample_nodes":
            out[key] = np.array([int(v) for v in rest], dtype=np.int64)
        elif key == "mesh_fingerprint":
            out[key] = rest[0]
        else:
            out[key] = float(rest[0]) if any(c in rest[0] for c in ".e") else int(rest[0])
    return out


if __name__ == "__main__":
    main()
