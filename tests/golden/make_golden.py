"""Write reference values for the full-size workloads with the CPU oracle.

Calls only oracle/ (and the seeded input generator).  For each workload it
stores E_J = 2 Tr(D J) and E_K = Tr(D K) (closed-shell reading, see DESIGN),
the number of significant unique quartets, and every 97th element of J and
K in row-major order.  Run: python tests/golden/make_golden.py c1 c2
(about half an hour per workload on 8 cores).

c4 (256 molecules, 4 densities each) stores, per molecule, both energies
for every density and every 2003rd element of J and K:
python tests/golden/make_golden.py c4 (about half an hour on 8 cores).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle as o  # noqa: E402
from paper_2507_09772_amd import synth  # noqa: E402

STRIDE = 97
BATCH_STRIDE = 2003


def batch_golden():
    mols = []
    t0 = time.time()
    for m, wl in enumerate(synth.batch_workload()):
        J, K, nsig = o.jk(wl.mol, wl.D, 1e-13, mode=1)
        ej, ek = o.energies(wl.D, J, K)
        mols.append(dict(nao=int(wl.mol.nao), nsig=nsig, E_J=[float(x) for x in ej], E_K=[float(x) for x in ek],
                         J=J.ravel()[::BATCH_STRIDE].tolist(), K=K.ravel()[::BATCH_STRIDE].tolist()))
        print(m, wl.mol.nwater, wl.mol.nao, f"{time.time() - t0:.0f}s", flush=True)
    out = dict(workload="c4", cutoff=1e-13, stride=BATCH_STRIDE, molecules=mols,
               oracle_seconds=time.time() - t0, oracle_threads=o.num_threads())
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_jk.json"), "w") as f:
        json.dump(out, f)


def main(names):
    o.build_oracle(force=False)
    for name in names:
        if name == "c4":
            batch_golden()
            continue
        wl = synth.workload(name)
        t0 = time.time()
        Q = o.schwarz(wl.mol)
        J, K, nsig = o.jk(wl.mol, wl.D, wl.cutoff, mode=1, Q=Q)
        dt = time.time() - t0
        ej, ek = o.energies(wl.D, J, K)
        out = dict(workload=name, nao=int(wl.mol.nao), cutoff=wl.cutoff, nsig=nsig,
                   E_J=float(ej[0]), E_K=float(ek[0]), stride=STRIDE,
                   J=J.ravel()[::STRIDE].tolist(), K=K.ravel()[::STRIDE].tolist(),
                   oracle_seconds=dt, oracle_threads=o.num_threads())
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_jk.json")
        with open(path, "w") as f:
            json.dump(out, f)
        print(name, "E_J", ej[0], "E_K", ek[0], "nsig", nsig, f"{dt:.0f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2"])
