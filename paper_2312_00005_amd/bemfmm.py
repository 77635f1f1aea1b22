"""ctypes binding of libbemfmm.so (include/bemfmm.h).

Argument marshalling only: every computation runs in the HIP library.  The
module-level ``bem_*`` functions mirror the C entry points one to one (same
names, same arguments, pointers as Python ints) and raise ``BemError`` on a
non-zero status.  ``Mesh`` wraps them for torch tensors: device buffers are
``torch.complex128`` tensors on the current HIP device and streams are
``torch.cuda.current_stream()``.

Importing this module fails loudly if the library has not been built.
"""

import ctypes
import os

# torch ships its own HIP runtime (soname libamdhip64.so.7).  Importing torch
# first makes the library below bind to that same runtime instead of loading a
# second copy from /opt/rocm, so both share one device context.
import torch  # noqa: F401

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbemfmm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2312_00005_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

BEM_OK, BEM_E_ARG, BEM_E_MESH, BEM_E_NOCONV, BEM_E_HIP, BEM_E_OOM, BEM_E_STATE = range(7)
BEM_PREC_FP64, BEM_PREC_MIXED = 0, 1
BEM_OP_A, BEM_OP_AH = 0, 1
BEM_WARN_COARSE_MESH, BEM_WARN_LARGE_L, BEM_WARN_NOT_CONVERGED = 1, 2, 4

_STATUS_NAMES = {0: "BEM_OK", 1: "BEM_E_ARG", 2: "BEM_E_MESH", 3: "BEM_E_NOCONV",
                 4: "BEM_E_HIP", 5: "BEM_E_OOM", 6: "BEM_E_STATE"}


class BemError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class bem_c128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class bem_options(ctypes.Structure):
    _fields_ = [
        ("use_fmm", ctypes.c_int32), ("levels", ctypes.c_int32), ("leaf_size", ctypes.c_int32),
        ("root_box_edge", ctypes.c_double), ("admissibility", ctypes.c_double),
        ("l_mode", ctypes.c_int32), ("l_factor", ctypes.c_double), ("l_min", ctypes.c_int32),
        ("l_eps", ctypes.c_double), ("t_order", ctypes.c_int32), ("quad_eps", ctypes.c_double),
        ("quad_m_max", ctypes.c_int32), ("quad_split_on_cap", ctypes.c_int32),
        ("subdiv_ratio", ctypes.c_double), ("max_subdiv", ctypes.c_int32),
        ("self_n", ctypes.c_int32), ("edge_parts", ctypes.c_int32), ("edge_gauss", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("gmres_restart", ctypes.c_int32),
        ("gmres_maxit", ctypes.c_int32), ("gmres_tol", ctypes.c_double),
        ("refine_maxit", ctypes.c_int32), ("inner_tol", ctypes.c_double),
        ("l_eps_mixed", ctypes.c_double), ("precond", ctypes.c_int32),
        ("gamma_re", ctypes.c_double), ("gamma_im_k", ctypes.c_double),
        ("far_direct", ctypes.c_int32), ("use_graphs", ctypes.c_int32), ("level_rows", ctypes.c_int32),
        ("solver", ctypes.c_int32), ("near_waves_per_cu", ctypes.c_int32),
        ("quad_eps_mixed", ctypes.c_double), ("interior", ctypes.c_int32),
        ("translate_shape", ctypes.c_int32), ("near_split", ctypes.c_int32),
        ("far_rows", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class bem_solve_info(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32), ("refinements", ctypes.c_int32), ("levels", ctypes.c_int32),
        ("L", ctypes.c_int32 * 16), ("clusters", ctypes.c_int32 * 16),
        ("near_pairs", ctypes.c_int64), ("near_items", ctypes.c_int64),
        ("quad_points", ctypes.c_int64), ("rel_residual", ctypes.c_double),
        ("warnings", ctypes.c_uint32), ("L_mixed", ctypes.c_int32 * 16),
    ]

    def as_dict(self):
        nl = self.levels
        return {"iterations": self.iterations, "refinements": self.refinements, "levels": nl,
                "L": list(self.L[:nl]), "L_mixed": list(self.L_mixed[:nl]),
                "clusters": list(self.clusters[:nl]),
                "near_pairs": self.near_pairs, "near_items": self.near_items,
                "quad_points": self.quad_points, "rel_residual": self.rel_residual,
                "warnings": self.warnings}


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double

_SIGS = {
    "bem_options_default": (_i32, [ctypes.POINTER(bem_options), ctypes.c_char_p]),
    "bem_mesh_create": (_i32, [_i64, _vp, _i64, _vp, ctypes.POINTER(bem_options), _vp, ctypes.POINTER(_vp)]),
    "bem_mesh_create_from_tree": (_i32, [_vp, ctypes.POINTER(bem_options), _vp, ctypes.POINTER(_vp)]),
    "bem_mesh_create_elements": (_i32, [_i64, _vp, _i64, _vp, ctypes.POINTER(bem_options), _vp,
                                        ctypes.POINTER(_vp)]),
    "bem_set_allocator": (_i32, [_vp, _vp, _vp]),
    "bem_mesh_bad_element": (_i64, [_vp]),
    "bem_set_problem": (_i32, [_vp, _dbl, _vp, _vp]),
    "bem_rhs_plane_wave": (_i32, [_vp, _vp, bem_c128, _vp, _vp]),
    "bem_rhs_point_source": (_i32, [_vp, _vp, bem_c128, _vp, _vp]),
    "bem_apply": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "bem_apply_part": (_i32, [_vp, _i32, _i32, _i32, _vp, _vp, _vp]),
    "bem_solve": (_i32, [_vp, _vp, _vp, _vp, _dbl, ctypes.POINTER(bem_solve_info), _vp]),
    "bem_apply_dc": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "bem_rhs_velocity": (_i32, [_vp, _vp, _dbl, _vp, _vp]),
    "bem_set_pressure_elements": (_i32, [_vp, _i64, _vp, _vp]),
    "bem_rhs_pressure": (_i32, [_vp, _vp, _vp, _vp]),
    "bem_incident_field": (_i32, [_vp, _i32, _vp, bem_c128, _i64, _vp, _vp, _vp]),
    "bem_autotune": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "bem_field": (_i32, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "bem_field_pv": (_i32, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "bem_field_noalloc": (_i32, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "bem_field_adjoint": (_i32, [_vp, _i64, _vp, _vp, _i32, _vp, _vp]),
    "bem_grad_admittance": (_i32, [_vp, _vp, _vp, _vp, _dbl, _vp, _vp]),
    "bem_solve_adjoint": (_i32, [_vp, _vp, _vp, ctypes.POINTER(bem_solve_info), _vp]),
    "bem_solve_batch": (_i32, [_i32, _vp, _vp, _vp, _vp, _dbl, _vp, _vp]),
    "bem_mesh_stats": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "bem_mesh_launch_shapes": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "bem_workspace_bytes": (ctypes.c_size_t, [_vp]),
    "bem_mesh_destroy": (None, [_vp]),
    "bem_last_error": (ctypes.c_char_p, []),
    "bem_tree_build": (_i32, [_i64, _vp, _i64, _vp, ctypes.POINTER(bem_options), ctypes.POINTER(_vp)]),
    "bem_tree_levels": (_i32, [_vp]),
    "bem_tree_level": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "bem_tree_level_data": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "bem_tree_perm": (_i32, [_vp, _vp]),
    "bem_tree_plan_stats": (_i32, [_vp, _vp, _vp, _vp]),
    "bem_tree_fmm_lengths": (_i32, [_vp, _dbl, ctypes.POINTER(bem_options), _vp, _vp, _vp, _vp]),
    "bem_tree_destroy": (None, [_vp]),
    "bem_mesh_diameter": (_i32, [_i64, _vp, _vp]),
    "bem_grid_create": (_i32, [_vp, _i64, _vp, ctypes.POINTER(_vp)]),
    "bem_grid_eval": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "bem_grid_stats": (_i32, [_vp, _vp, _vp, _vp]),
    "bem_grid_destroy": (None, [_vp]),
    "bem_auto_method": (_i32, [_i32, _i64, _dbl, _dbl, _vp]),
}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def exported_symbols():
    return sorted(_SIGS)


def _check(status):
    if status != BEM_OK:
        msg = _lib.bem_last_error()
        raise BemError(status, msg.decode() if msg else "")
    return status


# ---- one-to-one wrappers of the C entry points -------------------------------

def bem_options_default(preset="paper"):
    o = bem_options()
    _check(_lib.bem_options_default(ctypes.byref(o), preset.encode()))
    return o


def bem_mesh_create_elements(n_nodes, xyz_ptr, n_el, el_ptr, options, stream=None):
    out = _vp()
    st = _lib.bem_mesh_create_elements(n_nodes, xyz_ptr, n_el, el_ptr, ctypes.byref(options), stream,
                                       ctypes.byref(out))
    _check(st)
    return out


def bem_mesh_create_from_tree(tree, options, stream=None):
    out = _vp()
    st = _lib.bem_mesh_create_from_tree(tree, ctypes.byref(options), stream, ctypes.byref(out))
    _check(st)
    return out


def bem_mesh_create(n_nodes, xyz_ptr, n_tri, tri_ptr, options, stream=None):
    out = _vp()
    st = _lib.bem_mesh_create(n_nodes, xyz_ptr, n_tri, tri_ptr, ctypes.byref(options), stream, ctypes.byref(out))
    _check(st)
    return out.value


BEM_ALLOC_FN = ctypes.CFUNCTYPE(_vp, ctypes.c_size_t, _vp)
BEM_FREE_FN = ctypes.CFUNCTYPE(None, _vp, ctypes.c_size_t, _vp)
_allocator_refs = []  # the callbacks must outlive every buffer allocated through them


def bem_set_allocator(alloc_fn, free_fn, ctx=None):
    """alloc_fn / free_fn: BEM_ALLOC_FN / BEM_FREE_FN instances, or both None
    (hipMalloc / hipFree)."""
    _check(_lib.bem_set_allocator(ctypes.cast(alloc_fn, _vp) if alloc_fn else None,
                                  ctypes.cast(free_fn, _vp) if free_fn else None, ctx))
    if alloc_fn:
        _allocator_refs.append((alloc_fn, free_fn))


def use_torch_allocator():
    """Back the library's device memory by PyTorch's caching allocator on the
    current device (torch.cuda.caching_allocator_alloc / _delete)."""
    torch = _torch()

    def _alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except Exception:  # out of memory: the library reports BEM_E_OOM
            return None

    def _free(ptr, nbytes, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    bem_set_allocator(BEM_ALLOC_FN(_alloc), BEM_FREE_FN(_free))


def use_hip_allocator():
    """Back the library's device memory by hipMalloc / hipFree again."""
    bem_set_allocator(None, None)


def bem_mesh_bad_element(mesh):
    return _lib.bem_mesh_bad_element(mesh)


def bem_set_problem(mesh, k, beta_ptr, stream):
    _check(_lib.bem_set_problem(mesh, k, beta_ptr, stream))


def bem_rhs_plane_wave(mesh, d, P0, rhs_ptr, stream):
    dd = (ctypes.c_double * 3)(*d)
    _check(_lib.bem_rhs_plane_wave(mesh, dd, bem_c128(P0.real, P0.imag), rhs_ptr, stream))


def bem_rhs_point_source(mesh, x0, P0, rhs_ptr, stream):
    xx = (ctypes.c_double * 3)(*x0)
    _check(_lib.bem_rhs_point_source(mesh, xx, bem_c128(P0.real, P0.imag), rhs_ptr, stream))


def bem_apply(mesh, op, prec, x_ptr, y_ptr, stream):
    _check(_lib.bem_apply(mesh, op, prec, x_ptr, y_ptr, stream))


def bem_apply_part(mesh, op, prec, part, x_ptr, y_ptr, stream):
    _check(_lib.bem_apply_part(mesh, op, prec, part, x_ptr, y_ptr, stream))


def bem_apply_dc(mesh, op, prec, x_ptr, y_ptr, stream):
    _check(_lib.bem_apply_dc(mesh, op, prec, x_ptr, y_ptr, stream))


def bem_rhs_velocity(mesh, u_ptr, rho_c, rhs_ptr, stream):
    _check(_lib.bem_rhs_velocity(mesh, u_ptr, float(rho_c), rhs_ptr, stream))


def bem_set_pressure_elements(mesh, n, elems_ptr, stream):
    _check(_lib.bem_set_pressure_elements(mesh, n, elems_ptr, stream))


def bem_rhs_pressure(mesh, pbar_ptr, rhs_ptr, stream):
    _check(_lib.bem_rhs_pressure(mesh, pbar_ptr, rhs_ptr, stream))


def bem_mesh_launch_shapes(mesh):
    w, t, nw, sp = ((_i32 * 2)() for _ in range(4))
    _check(_lib.bem_mesh_launch_shapes(mesh, w, t, nw, sp))
    return {"near_wpb": {"fp64": w[0], "mixed": w[1]}, "translate_tpb": {"fp64": t[0], "mixed": t[1]},
            "near_waves_per_cu": {"fp64": nw[0], "mixed": nw[1]}, "near_split": {"fp64": sp[0], "mixed": sp[1]}}


def bem_autotune(mesh, stream):
    w = (_i32 * 2)()
    t = (_i32 * 2)()
    nw = (_i32 * 2)()
    _check(_lib.bem_autotune(mesh, w, t, nw, stream))
    return bem_mesh_launch_shapes(mesh)


def bem_incident_field(mesh, kind, src, P0, n_pts, pts_ptr, out_ptr, stream):
    s3 = (ctypes.c_double * 3)(*[float(v) for v in src])
    _check(_lib.bem_incident_field(mesh, int(kind), s3, bem_c128(P0.real, P0.imag), n_pts, pts_ptr, out_ptr,
                                   stream))


def bem_field(mesh, n_pts, pts_ptr, p_ptr, pinc_ptr, out_ptr, energy_ptr, stream):
    _check(_lib.bem_field(mesh, n_pts, pts_ptr, p_ptr, pinc_ptr, out_ptr, energy_ptr, stream))


def bem_field_noalloc(mesh, n_pts, pts_ptr, p_ptr, pinc_ptr, out_ptr, energy_ptr, stream):
    _check(_lib.bem_field_noalloc(mesh, n_pts, pts_ptr, p_ptr, pinc_ptr, out_ptr, energy_ptr, stream))


def bem_field_pv(mesh, n_pts, pts_ptr, p_ptr, dpdn_ptr, pinc_ptr, out_ptr, energy_ptr, stream):
    _check(_lib.bem_field_pv(mesh, n_pts, pts_ptr, p_ptr, dpdn_ptr, pinc_ptr, out_ptr, energy_ptr, stream))


def bem_field_adjoint(mesh, n_pts, pts_ptr, g_ptr, part, y_ptr, stream):
    _check(_lib.bem_field_adjoint(mesh, n_pts, pts_ptr, g_ptr, part, y_ptr, stream))


def bem_grad_admittance(mesh, p_ptr, w_ptr, hg_ptr, rho_c, grad_ptr, stream):
    _check(_lib.bem_grad_admittance(mesh, p_ptr, w_ptr, hg_ptr, rho_c, grad_ptr, stream))


def bem_solve_adjoint(mesh, rhs_ptr, x_ptr, stream):
    info = bem_solve_info()
    st = _lib.bem_solve_adjoint(mesh, rhs_ptr, x_ptr, ctypes.byref(info), stream)
    return st, info


def bem_solve(mesh, rhs_ptr, p_ptr, v_ptr, rho_c, stream):
    info = bem_solve_info()
    st = _lib.bem_solve(mesh, rhs_ptr, p_ptr, v_ptr, rho_c, ctypes.byref(info), stream)
    return st, info


def bem_solve_batch(meshes, rhs_ptrs, p_ptrs, v_ptrs, rho_c, stream):
    """meshes: mesh handles; rhs_ptrs, p_ptrs: device pointers; v_ptrs: None
    or a list of device pointers / None.  Returns (status, [bem_solve_info])."""
    n = len(meshes)
    arr = lambda vals: (_vp * max(n, 1))(*[v if v else None for v in vals]) if n else None
    infos = (bem_solve_info * max(n, 1))()
    st = _lib.bem_solve_batch(n, arr(meshes), arr(rhs_ptrs), arr(p_ptrs),
                              arr(v_ptrs) if v_ptrs is not None else None, float(rho_c or 0.0),
                              ctypes.cast(infos, _vp), stream)
    return st, [infos[i] for i in range(n)]


def bem_mesh_stats(mesh):
    lv = _i32()
    cl = (_i32 * 16)()
    npairs, nitems, npts = _i64(), _i64(), _i64()
    _check(_lib.bem_mesh_stats(mesh, ctypes.byref(lv), cl, ctypes.byref(npairs), ctypes.byref(nitems),
                               ctypes.byref(npts)))
    return {"levels": lv.value, "clusters": list(cl[:lv.value]), "near_pairs": npairs.value,
            "near_items": nitems.value, "quad_points": npts.value}


def bem_workspace_bytes(mesh):
    return _lib.bem_workspace_bytes(mesh)


def bem_mesh_destroy(mesh):
    _lib.bem_mesh_destroy(mesh)


def bem_last_error():
    m = _lib.bem_last_error()
    return m.decode() if m else ""


def bem_tree_build(n_nodes, xyz_ptr, n_tri, tri_ptr, options):
    out = _vp()
    _check(_lib.bem_tree_build(n_nodes, xyz_ptr, n_tri, tri_ptr, ctypes.byref(options), ctypes.byref(out)))
    return out.value


def bem_tree_levels(tree):
    return _lib.bem_tree_levels(tree)


def bem_tree_level(tree, level):
    nc, nil, nnr = _i64(), _i64(), _i64()
    _check(_lib.bem_tree_level(tree, level, ctypes.byref(nc), ctypes.byref(nil), ctypes.byref(nnr)))
    return nc.value, nil.value, nnr.value


def bem_tree_level_data(tree, level):
    import numpy as np
    nc, nil, nnr = bem_tree_level(tree, level)
    out = {"z": np.zeros((nc, 3)), "r": np.zeros(nc), "ebeg": np.zeros(nc, np.int64),
           "eend": np.zeros(nc, np.int64), "parent": np.zeros(nc, np.int64),
           "il_off": np.zeros(nc + 1, np.int64), "il": np.zeros(max(nil, 1), np.int64),
           "near_off": np.zeros(nc + 1, np.int64), "near": np.zeros(max(nnr, 1), np.int64)}
    p = {k_: v.ctypes.data for k_, v in out.items()}
    _check(_lib.bem_tree_level_data(tree, level, p["z"], p["r"], p["ebeg"], p["eend"], p["parent"],
                                    p["il_off"], p["il"], p["near_off"], p["near"]))
    out["il"] = out["il"][:nil]
    out["near"] = out["near"][:nnr]
    return out


def bem_tree_perm(tree, n_tri):
    import numpy as np
    perm = np.zeros(n_tri, np.int64)
    _check(_lib.bem_tree_perm(tree, perm.ctypes.data))
    return perm


def bem_tree_plan_stats(tree):
    a, b_, c = _i64(), _i64(), _i64()
    _check(_lib.bem_tree_plan_stats(tree, ctypes.byref(a), ctypes.byref(b_), ctypes.byref(c)))
    return {"near_pairs": a.value, "near_items": b_.value, "quad_points": c.value}


def bem_tree_destroy(tree):
    _lib.bem_tree_destroy(tree)


BEM_METHOD_BEM, BEM_METHOD_SLFMM, BEM_METHOD_MLFMM = 0, 1, 4


def bem_mesh_diameter(nodes):
    """Largest distance between two nodes (host array of shape (n, 3))."""
    import numpy as np
    xyz = np.ascontiguousarray(nodes, dtype=np.float64)
    d = _dbl()
    _check(_lib.bem_mesh_diameter(xyz.shape[0], xyz.ctypes.data, ctypes.byref(d)))
    return d.value


def bem_auto_method(requested, n_tri, diameter, k):
    out = _i32()
    _check(_lib.bem_auto_method(int(requested), int(n_tri), float(diameter), float(k), ctypes.byref(out)))
    return out.value


def bem_tree_fmm_lengths(tree, k, options):
    nl = bem_tree_levels(tree)
    L = (_i32 * 16)()
    L32 = (_i32 * 16)()
    capped = _i32()
    nbytes = _dbl()
    _check(_lib.bem_tree_fmm_lengths(tree, float(k), ctypes.byref(options), L, L32, ctypes.byref(capped),
                                     ctypes.byref(nbytes)))
    return {"L": list(L[:nl]), "L_mixed": list(L32[:nl]), "capped": bool(capped.value),
            "capped_fp64": bool(capped.value & 1), "capped_mixed": bool(capped.value & 2), "bytes": nbytes.value}


def bem_grid_create(mesh, pts):
    import numpy as np
    xyz = np.ascontiguousarray(pts, dtype=np.float64)
    out = _vp()
    _check(_lib.bem_grid_create(mesh, xyz.shape[0], xyz.ctypes.data, ctypes.byref(out)))
    return out.value


def bem_grid_eval(grid, p_ptr, dpdn_ptr, pinc_ptr, out_ptr, energy_ptr, stream):
    _check(_lib.bem_grid_eval(grid, p_ptr, dpdn_ptr, pinc_ptr, out_ptr, energy_ptr, stream))


def bem_grid_stats(grid):
    a, b, c = _i64(), _i64(), _i64()
    _check(_lib.bem_grid_stats(grid, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return {"point_clusters": a.value, "far_pairs": b.value, "near_elements": c.value}


def bem_grid_destroy(grid):
    _lib.bem_grid_destroy(grid)


class Grid:
    """Evaluation grid (bem_grid_*) of a Mesh: pressure at many field points
    with the far part from the FMM."""

    def __init__(self, mesh, pts):
        import numpy as np
        self.mesh = mesh  # the grid keeps a pointer to the mesh
        self.n = int(np.asarray(pts).shape[0])
        self._h = None
        self._h = bem_grid_create(mesh.handle, pts)

    def eval(self, p_surf, dpdn_surf=None, p_inc=None, energy=False):
        torch = _torch()
        out = self.mesh._empty(self.n)
        en = torch.zeros((), dtype=torch.float64, device="cuda") if energy else None
        bem_grid_eval(self._h, _dev_c128(p_surf, self.mesh.n, "p_surf"),
                      _dev_c128(dpdn_surf, self.mesh.n, "dpdn_surf") if dpdn_surf is not None else None,
                      _dev_c128(p_inc, self.n, "p_inc") if p_inc is not None else None, out.data_ptr(),
                      en.data_ptr() if en is not None else None, _stream())
        return (out, en) if energy else out

    def stats(self):
        return bem_grid_stats(self._h)

    def close(self):
        if self._h:
            bem_grid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HostTree:
    """Host-only cluster tree and near-field plan (no GPU needed)."""

    def __init__(self, nodes, tris, options=None, **overrides):
        import numpy as np
        if options is None or isinstance(options, str):
            options = bem_options_default(options or "paper")
        for key, val in overrides.items():
            setattr(options, key, val)
        self._nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        self._tris = np.ascontiguousarray(tris, dtype=np.int32)
        self.n = int(self._tris.shape[0])
        self._h = None
        self.options = options
        self._h = bem_tree_build(self._nodes.shape[0], self._nodes.ctypes.data, self.n,
                                 self._tris.ctypes.data, options)

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                bem_tree_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def levels(self):
        return [bem_tree_level_data(self._h, l) for l in range(bem_tree_levels(self._h))]

    def perm(self):
        return bem_tree_perm(self._h, self.n)

    def plan_stats(self):
        return bem_tree_plan_stats(self._h)

    def fmm_lengths(self, k):
        """Expansion lengths at wavenumber k, whether the stability cap lowered
        any, and the estimated far-field device bytes."""
        return bem_tree_fmm_lengths(self._h, k, self.options)


# ---- torch convenience layer -------------------------------------------------

def _torch():
    import torch
    return torch


def _stream():
    """The current torch stream, or None (the default stream) where torch has
    no device: the host-side checks of every entry point run before any
    device work, so argument errors are reported without a GPU."""
    torch = _torch()
    if not torch.cuda.is_available():
        return None
    return torch.cuda.current_stream().cuda_stream


def _dev_c128(t, n, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 device tensor")
    if t.numel() != n or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous with {n} elements")
    return t.data_ptr()


def _dev_pts(pts):
    torch = _torch()
    if not isinstance(pts, torch.Tensor) or pts.dtype != torch.float64 or not pts.is_cuda \
            or pts.dim() != 2 or pts.shape[1] != 3:
        raise TypeError("pts must be a float64 device tensor of shape (n, 3)")
    return pts.contiguous()


_PRECS = {"fp64": BEM_PREC_FP64, "mixed": BEM_PREC_MIXED, BEM_PREC_FP64: BEM_PREC_FP64,
          BEM_PREC_MIXED: BEM_PREC_MIXED}
_OPS = {"A": BEM_OP_A, "AH": BEM_OP_AH, BEM_OP_A: BEM_OP_A, BEM_OP_AH: BEM_OP_AH}


class Mesh:
    """A bem_mesh with torch-tensor helpers.  Elements keep the caller's order."""

    def __init__(self, nodes, tris, options=None, **overrides):
        import numpy as np
        if options is None:
            options = bem_options_default("paper")
        elif isinstance(options, str):
            options = bem_options_default(options)
        for key, val in overrides.items():
            setattr(options, key, val)
        self.options = options
        self._nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        self._tris = np.ascontiguousarray(tris, dtype=np.int32)
        self.n = int(self._tris.shape[0])
        self._h = None
        if self._tris.ndim != 2 or self._tris.shape[1] not in (3, 4):
            raise ValueError("elements must be an (n, 3) or (n, 4) index array")
        # (n, 4): triangles and plane quadrilaterals (-1 in the last column of a triangle)
        create = bem_mesh_create if self._tris.shape[1] == 3 else bem_mesh_create_elements
        self._h = create(self._nodes.shape[0], self._nodes.ctypes.data, self.n, self._tris.ctypes.data, options,
                         _stream())
        self._beta = None

    @classmethod
    def from_tree(cls, tree, options=None, **overrides):
        """A mesh on a HostTree's geometry, tree and near plan (built once in
        the tree and copied): options default to the tree's, with overrides;
        the tree and plan fields must stay the tree's."""
        m = cls.__new__(cls)
        m._h = None
        if options is None:
            options = bem_options.from_buffer_copy(tree.options)
        elif isinstance(options, str):
            options = bem_options_default(options)
        for key, val in overrides.items():
            setattr(options, key, val)
        m.options = options
        m._nodes, m._tris, m.n = tree._nodes, tree._tris, tree.n
        m._beta = None
        m._h = bem_mesh_create_from_tree(tree._h, options, _stream())
        return m

    def close(self):
        if self._h:
            bem_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_problem(self, k, beta=None):
        ptr = None
        if beta is not None:
            ptr = _dev_c128(beta, self.n, "beta")
            self._beta = beta
        bem_set_problem(self._h, float(k), ptr, _stream())

    def _empty(self, n=None):
        torch = _torch()
        return torch.empty(self.n if n is None else n, dtype=torch.complex128, device="cuda")

    def rhs_plane_wave(self, d=(0.0, 0.0, 1.0), P0=1.0):
        out = self._empty()
        bem_rhs_plane_wave(self._h, d, complex(P0), out.data_ptr(), _stream())
        return out

    def rhs_point_source(self, x0, P0=1.0):
        out = self._empty()
        bem_rhs_point_source(self._h, x0, complex(P0), out.data_ptr(), _stream())
        return out

    def apply(self, x, op="A", prec="fp64", out=None):
        xp = _dev_c128(x, self.n, "x")
        out = self._empty() if out is None else out
        bem_apply(self._h, _OPS[op], _PRECS[prec], xp, _dev_c128(out, self.n, "y"), _stream())
        return out

    def apply_part(self, x, part, op="A", prec="fp64", out=None):
        """part 1: diagonal + near field only; part 2: far field only."""
        xp = _dev_c128(x, self.n, "x")
        out = self._empty() if out is None else out
        bem_apply_part(self._h, _OPS[op], _PRECS[prec], int(part), xp, _dev_c128(out, self.n, "y"),
                       _stream())
        return out

    def apply_dc(self, x, op="A", prec="fp64", out=None):
        """y = V x (or V^H x), V = dA/dc."""
        xp = _dev_c128(x, self.n, "x")
        out = self._empty() if out is None else out
        bem_apply_dc(self._h, _OPS[op], _PRECS[prec], xp, _dev_c128(out, self.n, "y"), _stream())
        return out

    def set_pressure_elements(self, elems):
        """PRES elements (host integer indices); their unknown becomes dp/dn.
        Call set_problem afterwards."""
        import numpy as np
        idx = np.ascontiguousarray(np.asarray(elems, dtype=np.int64).ravel())
        bem_set_pressure_elements(self._h, idx.size, idx.ctypes.data if idx.size else None, _stream())

    def rhs_add_pressure(self, rhs, pbar):
        """rhs -= A pbar over the PRES elements, in place."""
        bem_rhs_pressure(self._h, _dev_c128(pbar, self.n, "pbar"), _dev_c128(rhs, self.n, "rhs"), _stream())
        return rhs

    def rhs_add_velocity(self, rhs, u, rho_c):
        """rhs -= i k rho_c V u in place: prescribed normal velocities u (VELO)."""
        bem_rhs_velocity(self._h, _dev_c128(u, self.n, "u"), rho_c, _dev_c128(rhs, self.n, "rhs"), _stream())
        return rhs

    def autotune(self):
        """Time the launch-shape candidates on this problem and keep the fastest."""
        return bem_autotune(self._h, _stream())

    def incident_plane_wave(self, pts, d=(0.0, 0.0, 1.0), P0=1.0):
        pts = _dev_pts(pts)
        out = self._empty(pts.shape[0])
        bem_incident_field(self._h, 0, d, complex(P0), pts.shape[0], pts.data_ptr(), out.data_ptr(), _stream())
        return out

    def incident_point_source(self, pts, x0, P0=1.0):
        pts = _dev_pts(pts)
        out = self._empty(pts.shape[0])
        bem_incident_field(self._h, 1, x0, complex(P0), pts.shape[0], pts.data_ptr(), out.data_ptr(), _stream())
        return out

    def field(self, pts, p_surf, p_inc=None, energy=False):
        """Exterior pressure at field points pts (device float64 [n, 3]);
        with energy=True also sum |p|^2 as a device float64 tensor of shape ()."""
        torch = _torch()
        pts = _dev_pts(pts)
        npts = pts.shape[0]
        out = self._empty(npts)
        pinc = _dev_c128(p_inc, npts, "p_inc") if p_inc is not None else None
        en = torch.zeros((), dtype=torch.float64, device="cuda") if energy else None
        bem_field(self._h, npts, pts.data_ptr(), _dev_c128(p_surf, self.n, "p_surf"), pinc, out.data_ptr(),
                  en.data_ptr() if en is not None else None, _stream())
        return (out, en) if energy else out

    def field_pv(self, pts, p_surf, dpdn_surf, p_inc=None, energy=False):
        """Exterior pressure from the surface pressure and its normal
        derivative given separately (any boundary condition, PRES included)."""
        torch = _torch()
        pts = _dev_pts(pts)
        npts = pts.shape[0]
        out = self._empty(npts)
        pinc = _dev_c128(p_inc, npts, "p_inc") if p_inc is not None else None
        en = torch.zeros((), dtype=torch.float64, device="cuda") if energy else None
        bem_field_pv(self._h, npts, pts.data_ptr(), _dev_c128(p_surf, self.n, "p_surf"),
                     _dev_c128(dpdn_surf, self.n, "dpdn_surf"), pinc, out.data_ptr(),
                     en.data_ptr() if en is not None else None, _stream())
        return (out, en) if energy else out

    def field_adjoint(self, pts, g, part=0):
        """y = K^H g with K the field map (part 0) or its G part (part 1)."""
        pts = _dev_pts(pts)
        npts = pts.shape[0]
        out = self._empty()
        bem_field_adjoint(self._h, npts, pts.data_ptr(), _dev_c128(g, npts, "g"), int(part), out.data_ptr(),
                          _stream())
        return out

    def grad_admittance(self, p, w, hg, rho_c):
        torch = _torch()
        out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        bem_grad_admittance(self._h, _dev_c128(p, self.n, "p"), _dev_c128(w, self.n, "w"),
                            _dev_c128(hg, self.n, "hg"), float(rho_c), out.data_ptr(), _stream())
        return out

    def solve_adjoint(self, rhs, allow_noconv=False):
        """x with A^H x = rhs; returns (x, info dict)."""
        rp = _dev_c128(rhs, self.n, "rhs")
        x = self._empty()
        st, info = bem_solve_adjoint(self._h, rp, x.data_ptr(), _stream())
        if st != BEM_OK and not (allow_noconv and st == BEM_E_NOCONV):
            _check(st)
        return x, info.as_dict()

    def solve(self, rhs, rho_c=None, allow_noconv=False):
        """Returns (p, v or None, info dict)."""
        rp = _dev_c128(rhs, self.n, "rhs")
        p = self._empty()
        v = self._empty() if rho_c is not None else None
        st, info = bem_solve(self._h, rp, p.data_ptr(), v.data_ptr() if v is not None else None,
                             float(rho_c) if rho_c is not None else 0.0, _stream())
        if st != BEM_OK and not (allow_noconv and st == BEM_E_NOCONV):
            _check(st)
        return p, v, info.as_dict()

    def stats(self):
        return bem_mesh_stats(self._h)

    @staticmethod
    def solve_batch(meshes, rhs_list, rho_c=None, allow_noconv=False):
        """Solve one system per mesh with bem_solve_batch (lock-step GMRES);
        returns [(p, v or None, info dict)]."""
        ps = [m._empty() for m in meshes]
        vs = [m._empty() for m in meshes] if rho_c is not None else None
        rp = [_dev_c128(r, m.n, "rhs") for m, r in zip(meshes, rhs_list)]
        st, infos = bem_solve_batch([m._h for m in meshes], rp, [p.data_ptr() for p in ps],
                                    [v.data_ptr() for v in vs] if vs is not None else None, rho_c, _stream())
        if st != BEM_OK and not (allow_noconv and st == BEM_E_NOCONV):
            _check(st)
        return [(ps[i], vs[i] if vs is not None else None, infos[i].as_dict()) for i in range(len(meshes))]

    def workspace_bytes(self):
        return bem_workspace_bytes(self._h)
