"""Frequency sweep on one mesh.

For every frequency the far-field method is chosen from what the library
reports about each candidate cluster tree (bem_tree_fmm_lengths): the deepest
tree whose expansion lengths are not lowered by the stability cap (k X_min
large enough, Sec. 3.3.1), stay within the supported length and fit the
memory budget runs the FMM; otherwise the far field is evaluated by direct
quadrature (far_direct), which has no low-frequency breakdown and needs no
translation memory.  Frequencies that share a method share one device plan
(geometry, tree, near plan built once); with batch = B a group holds B
mesh instances and solves B frequencies at a time with bem_solve_batch, whose
lock-step GMRES keeps the device busy while each system's Gram-Schmidt
coefficients travel to the host.  Solving several frequencies concurrently
from several host threads (one HIP stream and mesh instance each) is
disabled: such a run ended once in a host segmentation fault inside the solve
whose cause has not been found.  Frequencies may come from a frequency-defining curve
(``FrequencySweep.from_curve``) and element groups may carry an admittance
that follows curves of the frequency step (``admittance=``, see curves.py);
each frequency is then solved with its own beta.  This module only schedules
calls into the library.
"""

import math
import time

from . import bemfmm, curves


def wavenumbers(freqs, c=343.0):
    return [2.0 * math.pi * f / c for f in freqs]


def paper_methods(nodes, tris, ks, requested=bemfmm.BEM_METHOD_MLFMM, depth=3):
    """Per wavenumber the method of the paper's automatic switches
    (bem_auto_method): ("dense", 0) for the conventional method, ("fmm", 1)
    for the single-level FMM, ("fmm", depth) for the multilevel FMM."""
    D = bemfmm.bem_mesh_diameter(nodes)
    out = []
    for k in ks:
        m = bemfmm.bem_auto_method(requested, len(tris), D, k)
        out.append(("dense", 0) if m == bemfmm.BEM_METHOD_BEM else
                   ("fmm", 1) if m == bemfmm.BEM_METHOD_SLFMM else ("fmm", depth))
    return out


def choose_methods(trees, ks, max_L=120, memory_budget=96e9, mixed=False):
    """Per wavenumber ("fmm", depth), ("fmm32", depth) or ("direct", depth);
    trees: {depth: HostTree}.  The deepest tree whose lengths stay within
    max_L and whose far-field memory fits is taken.  FP64 path: the FMM where
    the stability cap leaves the FP64 lengths intact, else the next depth, else
    the direct far field.  Mixed path (mixed=True): the FMM where the FP64
    lengths are intact; where they are capped, "fmm32": the complex-FP32 inner
    operator keeps its FMM (however its own lengths were capped: it only has
    to drive the inner solves, measured within 1e-5 of the direct far field at
    100-1000 Hz on the 40500-triangle sphere) and the FP64 operator of the
    refinement residuals integrates the far field directly, so the solution
    keeps the FP64 operator's accuracy."""
    out = []
    deepest = max(trees)
    for k in ks:
        pick = ("direct", deepest)
        for d in sorted(trees, reverse=True):
            info = trees[d].fmm_lengths(k)
            if info["bytes"] > memory_budget or max(info["L"] + info["L_mixed"]) > max_L:
                continue
            if not info["capped_fp64"] and (mixed or not info["capped"]):
                pick = ("fmm", d)
                break
            if mixed:
                pick = ("fmm32", d)
                break
        out.append(pick)
    return out


class FrequencySweep:
    """Solve the exterior problem at every frequency of ``freqs`` on one mesh."""

    def __init__(self, nodes, tris, freqs, c=343.0, preset="mixed", depths=(4, 3, 2), leaf_size=32,
                 memory_budget=96e9, max_L=120, streams=1, steps=None, admittance=None, rho=1.21, batch=1,
                 policy="stability", requested=bemfmm.BEM_METHOD_MLFMM, probe=True, **overrides):
        """policy: "stability" (the deepest tree whose expansion the stability
        cap leaves intact, else the direct far field) or "paper" (the paper's
        automatic switches between the conventional method, the single-level
        and the multilevel FMM, from the requested method).
        probe (mixed path, stability policy): before solving, the frequencies
        given "fmm32" (FP64 lengths shortened by the stability cap, FP64
        operator integrating the far field directly) are probed on the device:
        where the capped FP64 FMM applies the same operator as the direct far
        field to a tenth of the GMRES tolerance (relative l2 on a seeded
        vector), the FP64 operator keeps the FMM ("fmm")."""
        """steps / admittance: the frequency step s of every frequency and a
        list of curves.AdmittanceGroup; each frequency is then solved with
        beta = rho c Y(s) per element (Y = 0, sound hard, outside the groups)."""
        self.nodes, self.tris = nodes, tris
        self.freqs = list(freqs)
        self.admittance = list(admittance) if admittance else []
        self.steps = None if steps is None else [float(v) for v in steps]
        if self.admittance and (self.steps is None or len(self.steps) != len(self.freqs)):
            raise ValueError("frequency-dependent admittance needs the frequency step of every frequency")
        self.rho_c = float(rho) * float(c)
        self.ks = wavenumbers(self.freqs, c)
        self.preset = preset
        self.leaf_size = leaf_size
        self.overrides = overrides
        self.streams = max(1, int(streams))
        self.batch = max(1, int(batch))
        self.probe = bool(probe)
        self.probes = []
        self._spare = {}  # method -> a mesh made for the probe, reused by that method's group
        if self.streams > 1:
            raise NotImplementedError("concurrent frequencies from several host threads are disabled "
                                      "(a host crash was seen in that mode and its cause is not known)")
        t0 = time.perf_counter()
        # host trees by depth (their near plans are built when a mesh of that
        # depth is first made from them, and shared by its method groups)
        self.trees = {}
        if policy == "paper":
            self.methods = paper_methods(nodes, tris, self.ks, requested, max(depths))
            self.lengths = [None] * len(self.ks)
        elif policy == "stability":
            self.trees = {d: bemfmm.HostTree(nodes, tris, preset, levels=d, leaf_size=leaf_size, **overrides)
                          for d in depths}
            opts = bemfmm.bem_options_default(preset)
            for key, val in overrides.items():
                setattr(opts, key, val)
            mixed = opts.precision != 0
            self.methods = choose_methods(self.trees, self.ks, max_L=max_L, memory_budget=memory_budget, mixed=mixed)
            self.lengths = [self.trees[d].fmm_lengths(k) for (kind, d), k in zip(self.methods, self.ks)]
            used = {d for _, d in self.methods}
            self.trees = {d: t for d, t in self.trees.items() if d in used}
        else:
            raise ValueError(f"unknown policy {policy!r}")
        self.plan_seconds = time.perf_counter() - t0

    def _mesh(self, method):
        kind, d = method
        if kind == "dense":
            return bemfmm.Mesh(self.nodes, self.tris, self.preset, use_fmm=0, **self.overrides)
        far = {"direct": 1, "fmm32": 2}.get(kind, 0)
        if d in self.trees:
            return bemfmm.Mesh.from_tree(self.trees[d], far_direct=far)
        return bemfmm.Mesh(self.nodes, self.tris, self.preset, use_fmm=1, levels=d, leaf_size=self.leaf_size,
                           far_direct=far, **self.overrides)

    def _probe_capped(self):
        """Relabel "fmm32" frequencies as "fmm" where the capped FP64 FMM is
        as good as the direct far field for this solve: relative l2 difference
        of the two FP64 far fields on a seeded vector at most a tenth of the
        GMRES tolerance.  The cap shortens the expansion less as k grows, so
        within one depth the test is monotone in k: a binary search finds the
        lowest frequency that passes and every higher one passes with it."""
        import torch
        opts = bemfmm.bem_options_default(self.preset)
        for key, val in self.overrides.items():
            setattr(opts, key, val)
        tol = 0.1 * opts.gmres_tol
        by_depth = {}
        for i, (kind, d) in enumerate(self.methods):
            if kind == "fmm32" and d in self.trees:
                by_depth.setdefault(d, []).append(i)
        for d, idx in by_depth.items():
            idx = sorted(idx, key=lambda i: self.ks[i])
            mf = bemfmm.Mesh.from_tree(self.trees[d], far_direct=0)
            md = bemfmm.Mesh.from_tree(self.trees[d], far_direct=1)
            gen = torch.Generator().manual_seed(20231200)
            n = mf.n
            x = torch.complex(torch.randn(n, generator=gen, dtype=torch.float64),
                              torch.randn(n, generator=gen, dtype=torch.float64)).to("cuda")

            def passes(i):
                b = self.beta(i)
                for m in (mf, md):
                    m.set_problem(self.ks[i], b)
                y0 = mf.apply_part(x, 2, prec="fp64")
                y1 = md.apply_part(x, 2, prec="fp64")
                err = float(torch.linalg.norm(y0 - y1) / torch.linalg.norm(mf.apply(x, prec="fp64")))
                self.probes.append({"f": self.freqs[i], "depth": d, "rel_l2": err, "pass": err <= tol})
                return err <= tol

            lo, hi = 0, len(idx)
            while lo < hi:
                mid = (lo + hi) // 2
                if passes(idx[mid]):
                    hi = mid
                else:
                    lo = mid + 1
            for i in idx[lo:]:
                self.methods[i] = ("fmm", d)
            # the two meshes serve the "fmm" and "direct" groups of this depth
            for key, mesh in ((("fmm", d), mf), (("direct", d), md)):
                if key in self._spare:
                    mesh.close()
                else:
                    self._spare[key] = mesh

    @classmethod
    def from_curve(cls, nodes, tris, n_steps, stepsize, s0, freq_curve, **kw):
        """Frequencies f_n = freq_curve(s0 + stepsize n), n = 1 .. n_steps."""
        s = curves.steps(n_steps, stepsize, s0)
        return cls(nodes, tris, [freq_curve(v) for v in s], steps=s, **kw)

    def beta(self, i):
        """Device beta = rho c Y of frequency i, or None (sound hard)."""
        if not self.admittance:
            return None
        import torch
        y = curves.element_admittance(self.admittance, len(self.tris), self.steps[i])
        return torch.from_numpy(self.rho_c * y).to("cuda")

    def source_strength(self, i, P0, curve_re=None, curve_im=None):
        """P0 at frequency i: c1(s) Re P0 + i c2(s) Im P0 with the step's
        curves (the input description scales source strengths like
        admittances); without curves P0 itself."""
        if curve_re is None and curve_im is None:
            return complex(P0)
        if self.steps is None:
            raise ValueError("a frequency-dependent source strength needs the frequency step of every frequency")
        return curves.AdmittanceGroup(None, P0, curve_re, curve_im).value(self.steps[i])

    def run(self, source=("plane", (0.0, 0.0, 1.0), 1.0), keep_solutions=True, source_curves=(None, None)):
        """Returns a list of per-frequency dicts (k, method, info, seconds, of
        which setup_seconds set up the frequency and solve_seconds solve it, and
        the device solution p) plus timing totals.  source_curves: curves of
        the frequency step for the real and imaginary part of P0.  With
        batch = B, each method group holds B mesh instances: B frequencies are
        set up (one per mesh) and solved together by bem_solve_batch; a
        frequency's seconds are then its share of the batch."""
        import torch
        t0 = time.perf_counter()
        t_probe = 0.0
        if self.probe and any(m[0] == "fmm32" for m in self.methods):
            self._probe_capped()
            torch.cuda.synchronize()
            t_probe = time.perf_counter() - t0
        groups = {}
        for i, m in enumerate(self.methods):
            groups.setdefault(m, []).append(i)
        results = [None] * len(self.ks)
        t_setup = t_probe
        for method, idx in groups.items():
            # the expansion tables grow with k and a buffer is only reallocated
            # when it grows: from the highest k down, every frequency of the
            # group reuses the first one's device memory (allocating anew at
            # every step of an ascending sweep has cost up to 2 s a frequency
            # at ~40 GB, after earlier groups had freed theirs)
            idx = sorted(idx, key=lambda i: -self.ks[i])
            ts = time.perf_counter()
            meshes = [self._spare.pop(method) if j == 0 and method in self._spare else self._mesh(method)
                      for j in range(min(self.batch, len(idx)))]
            t_setup += time.perf_counter() - ts
            for c0 in range(0, len(idx), len(meshes)):
                chunk = idx[c0:c0 + len(meshes)]
                t1 = time.perf_counter()
                rhs = []
                for mesh, i in zip(meshes, chunk):
                    mesh.set_problem(self.ks[i], self.beta(i))
                    kind, src, P0 = source
                    P0 = self.source_strength(i, P0, *source_curves)
                    rhs.append(mesh.rhs_plane_wave(src, P0) if kind == "plane" else mesh.rhs_point_source(src, P0))
                torch.cuda.current_stream().synchronize()
                t2 = time.perf_counter()
                if len(chunk) == 1:
                    out = [meshes[0].solve(rhs[0], allow_noconv=True)]
                else:
                    out = bemfmm.Mesh.solve_batch(meshes[:len(chunk)], rhs, allow_noconv=True)
                torch.cuda.current_stream().synchronize()
                t3 = time.perf_counter()
                dt = (t3 - t1) / len(chunk)
                for (p, _, info), i in zip(out, chunk):
                    results[i] = {"f": self.freqs[i], "k": self.ks[i], "method": self.methods[i], "info": info,
                                  "seconds": dt, "setup_seconds": (t2 - t1) / len(chunk),
                                  "solve_seconds": (t3 - t2) / len(chunk), "p": p if keep_solutions else None}
            for mesh in meshes:
                mesh.close()
        for mesh in self._spare.values():
            mesh.close()
        self._spare = {}
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return results, {"wall_s": wall, "mesh_setup_s": t_setup, "probe_s": t_probe,
                         "plan_choice_s": self.plan_seconds, "solve_s_per_frequency": (wall - t_setup) / len(self.ks)}
