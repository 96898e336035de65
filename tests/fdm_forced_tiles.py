"""Helper of tests/test_gpu_fdm.py (run in a fresh process): the
fast-diagonalisation inverse with a transform tile shape forced through the
tuning cache, against the oracle's inverse.

    python tests/fdm_forced_tiles.py <cache file> <ntc>

Writes one cache line per case mesh selecting <ntc> column tiles on every
axis, points DG_TUNE_CACHE at the file before the library's first tuning
look-up, and prints one JSON line per case: {"case": ..., "rel": ...}."""
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import synth  # noqa: E402
from oracle import kron  # noqa: E402
from tests.helpers import make_spec, ndof  # noqa: E402

CASES = [((5, 3, 7), 7, (0, 0, 1), True, 30.0, 1.0),
         ((2, 3, 1), 8, (0, 1, 2), False, 0.5, 2.0),
         ((6, 1, 2), 3, (2, 0, 1), False, 4.0, 1.0),
         ((4, 4, 4), 4, (0, 0, 0), False, 1.0, 1.0)]


def main():
    cache, ntc = sys.argv[1], int(sys.argv[2])
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.replace(" ", "_")
    with open(cache, "w") as f:
        for n, P, bc, st, lam, nu in CASES:
            f.write("fdm %s %d %d %d %d %d %d %d\n" % (arch, P, n[0], n[1], n[2], ntc, ntc, ntc))
    os.environ["DG_TUNE_CACHE"] = cache
    import paper_2112_04167_amd as dg
    for case in CASES:
        n, P, bc, st, lam, nu = case
        spec = make_spec(n, P, bc, st)
        b = synth.uniform_field(ndof(spec), 90 + P)
        mesh = dg.mesh_from_spec(spec)
        bd = torch.from_numpy(b).to("cuda")
        xd = torch.full_like(bd, float("nan"))
        dg.helmholtz_fdm_apply(mesh, lam, nu, bd, xd)
        torch.cuda.synchronize()
        x = xd.cpu().numpy()
        mesh.destroy()
        xo = kron.FDM(spec, lam, nu).apply_inverse(b)
        rel = float(np.linalg.norm(x - xo) / np.linalg.norm(xo)) if np.all(np.isfinite(x)) else float("inf")
        print(json.dumps({"case": str(case[:3]), "rel": rel}), flush=True)


if __name__ == "__main__":
    main()
