"""Write tests/golden/c4_sphere40500.npz from the CPU oracle alone.

Workload: the frequency sweep's 40500-triangle geodesic sphere (frequency 45,
radius 1), rigid, in air (c = 343 m/s), the coupling and quadrature rules of
the ``mixed`` preset (the ``tight`` rules) with the order tolerance lowered to
1e-11 (converged quadrature), at three of the sweep's 64 frequencies
f_i = 100 * 200^(i/63) Hz: i = 0 (100 Hz), 27 (about 1 kHz) and 36 (about
2.1 kHz, six elements per wavelength on this mesh).

Stored per frequency i (caller's element order): p_lu_<i>, the LU solution
(LAPACK zgetrf / zgetrs, Sec. 3.2) of the plane-wave problem exp(ikz), and
b_<i>, its right-hand side.  The dense matrix (26.2 GB complex128) is
assembled into Fortran-ordered shared memory by one worker process per host
core and factored in place.  Run from the repository root:

    python tests/golden/make_c4_golden.py [--workers 8]

It imports only ``oracle`` and ``synth``; about 20 minutes per frequency on 8
cores and 30 GB of memory.
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
from oracle.geometry import element_geometry  # noqa: E402
from oracle.presets import preset  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_sphere40500.npz")
QUAD_EPS = 1e-11
FREQ = 45
INDICES = (0, 27, 36)
C_AIR = 343.0

_G = {}


def frequency(i):
    return 100.0 * 200.0 ** (i / 63.0)


def _init(shm_name, N, k, freq):
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    nodes, tris = synth.geodesic_sphere(freq)
    _G["geom"] = element_geometry(nodes, tris)
    _G["shm"] = shared_memory.SharedMemory(name=shm_name)
    _G["A"] = np.ndarray((N, N), dtype=np.complex128, buffer=_G["shm"].buf, order="F")
    _G["k"] = k
    _G["p"] = preset("mixed", quad_eps=QUAD_EPS)


def _rows(block):
    r0, r1 = block
    _G["A"][r0:r1, :] = op.rows(_G["geom"], np.arange(r0, r1), _G["k"], p=_G["p"])
    return r0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count())
    ap.add_argument("--block", type=int, default=64)
    ap.add_argument("--freq", type=int, default=FREQ, help="other sizes: dry runs only")
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()
    nodes, tris = synth.geodesic_sphere(args.freq)
    N = len(tris)
    g = element_geometry(nodes, tris)
    out = {"N": np.int64(N), "quad_eps": np.float64(QUAD_EPS), "indices": np.array(INDICES),
           "c": np.float64(C_AIR)}
    import scipy.linalg
    shm = shared_memory.SharedMemory(create=True, size=N * N * 16)
    try:
        for i in INDICES:
            f = frequency(i)
            k = 2.0 * math.pi * f / C_AIR
            A = np.ndarray((N, N), dtype=np.complex128, buffer=shm.buf, order="F")
            blocks = [(r, min(N, r + args.block)) for r in range(0, N, args.block)]
            t0 = time.perf_counter()
            with Pool(args.workers, initializer=_init, initargs=(shm.name, N, k, args.freq)) as pool:
                for n_done, _ in enumerate(pool.imap_unordered(_rows, blocks)):
                    if n_done % 64 == 0:
                        print(f"  f = {f:.1f} Hz: {n_done + 1}/{len(blocks)} blocks, "
                              f"{time.perf_counter() - t0:.0f} s", flush=True)
            t_asm = time.perf_counter() - t0
            b = op.rhs_plane_wave(g, k, [0.0, 0.0, 1.0], p=preset("mixed"))
            t0 = time.perf_counter()
            lu, piv = scipy.linalg.lu_factor(A, overwrite_a=True, check_finite=False)
            p_lu = scipy.linalg.lu_solve((lu, piv), b, check_finite=False)
            t_lu = time.perf_counter() - t0
            del lu, piv, A
            print(f"f = {f:.1f} Hz (k = {k:.4f}): assembly {t_asm:.0f} s, LU {t_lu:.0f} s", flush=True)
            out[f"p_lu_{i}"] = p_lu
            out[f"b_{i}"] = b
            out[f"k_{i}"] = np.float64(k)
            out[f"t_assembly_s_{i}"] = np.float64(t_asm)
            out[f"t_lu_s_{i}"] = np.float64(t_lu)
    finally:
        shm.close()
        shm.unlink()
    np.savez_compressed(args.out, **out)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
