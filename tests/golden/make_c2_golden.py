"""Write tests/golden/c2_sphere20480.npz from the CPU oracle alone.

Workload: the 20480-triangle icosphere (subdivision 5, radius 1), k for six
elements per wavelength (k = 2 pi / (6 h), h the mean edge length), rigid
surface, the coupling and quadrature rules of the ``tight`` preset with the
order tolerance lowered to 1e-11 (converged quadrature: the a-priori order
estimates of Sec. 3.1.4 at 1e-8 do not resolve the oscillation of exp(ikr) on
far elements, see Sec. 5.1.3 for the paper's own FMM-versus-direct
comparison).

Stored values (caller's element order):
  y_ax : A x with x = synth.complex_normal(N, seed=4), the full dense
         operator of Eq. (SystemI) applied to one seeded vector
  p_lu : the LU solution (LAPACK zgetrf / zgetrs, the paper's direct solver,
         Sec. 3.2) for the plane wave exp(ikz) (P0 = 1)
  b    : that right-hand side, b = p_inc - gamma dp_inc/dn (Sec. 2.4)

The dense matrix (6.7 GB complex128) is assembled row block by row block in
worker processes (one per host core) into shared memory and factored in
place.  Run from the repository root:

    python tests/golden/make_c2_golden.py [--workers 8]

It imports only ``oracle`` and ``synth``; about 10 minutes on 8 cores.
"""

import argparse
import math
import os
import sys
import time
from multiprocessing import Pool, shared_memory

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import operator as op  # noqa: E402
from oracle import sphere  # noqa: E402
from oracle.geometry import element_geometry  # noqa: E402
from oracle.presets import preset  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_sphere20480.npz")
QUAD_EPS = 1e-11
SUBDIV = 5
X_SEED = 4

_G = {}


def _init(shm_name, N, k, subdiv):
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    nodes, tris = synth.icosphere(subdiv)
    _G["geom"] = element_geometry(nodes, tris)
    _G["shm"] = shared_memory.SharedMemory(name=shm_name)
    _G["A"] = np.ndarray((N, N), dtype=np.complex128, buffer=_G["shm"].buf)
    _G["k"] = k
    _G["x"] = synth.complex_normal(N, seed=X_SEED)
    _G["p"] = preset("tight", quad_eps=QUAD_EPS)


def _rows(block):
    r0, r1 = block
    Ab = op.rows(_G["geom"], np.arange(r0, r1), _G["k"], p=_G["p"])
    _G["A"][r0:r1] = Ab
    return r0, Ab @ _G["x"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count())
    ap.add_argument("--block", type=int, default=64)
    ap.add_argument("--subdiv", type=int, default=SUBDIV, help="other sizes: dry runs only")
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()
    nodes, tris = synth.icosphere(args.subdiv)
    N = len(tris)
    k = 2.0 * math.pi / (6.0 * synth.mean_edge_length(nodes, tris))
    g = element_geometry(nodes, tris)
    x = synth.complex_normal(N, seed=X_SEED)
    shm = shared_memory.SharedMemory(create=True, size=N * N * 16)
    try:
        A = np.ndarray((N, N), dtype=np.complex128, buffer=shm.buf)
        blocks = [(r, min(N, r + args.block)) for r in range(0, N, args.block)]
        y = np.zeros(N, dtype=np.complex128)
        t0 = time.perf_counter()
        with Pool(args.workers, initializer=_init, initargs=(shm.name, N, k, args.subdiv)) as pool:
            for i, (r0, yb) in enumerate(pool.imap_unordered(_rows, blocks)):
                y[r0:r0 + yb.size] = yb
                if i % 32 == 0:
                    print(f"  rows: {i + 1}/{len(blocks)} blocks, {time.perf_counter() - t0:.0f} s", flush=True)
        t_asm = time.perf_counter() - t0
        print(f"assembled N = {N} (k = {k:.6f}) in {t_asm:.1f} s on {args.workers} processes", flush=True)
        b = op.rhs_plane_wave(g, k, [0.0, 0.0, 1.0], p=preset("tight"))
        t0 = time.perf_counter()
        import scipy.linalg
        lu = scipy.linalg.lu_factor(A, overwrite_a=True, check_finite=False)
        p_lu = scipy.linalg.lu_solve(lu, b, check_finite=False)
        t_lu = time.perf_counter() - t0
        del lu
        print(f"LU factor + solve {t_lu:.1f} s", flush=True)
    finally:
        A = None
        shm.close()
        shm.unlink()
    an = sphere.pressure(g["x"] / np.linalg.norm(g["x"], axis=1, keepdims=True), k)
    err_an = np.linalg.norm(p_lu - an) / np.linalg.norm(an)
    print(f"LU solution vs analytic rigid-sphere series: {err_an:.3e} (discretisation error)")
    np.savez_compressed(args.out, y_ax=y, p_lu=p_lu, b=b, k=np.float64(k), N=np.int64(N),
                        quad_eps=np.float64(QUAD_EPS), x_seed=np.int64(X_SEED),
                        gamma_im_k=np.float64(preset("tight")["gamma_im_k"]),
                        t_assembly_s=np.float64(t_asm), t_lu_s=np.float64(t_lu),
                        workers=np.int64(args.workers))
    print("wrote", args.out)


if __name__ == "__main__":
    main()
