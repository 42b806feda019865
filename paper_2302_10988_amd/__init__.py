"""MI355X travel-time solver for generally anisotropic media (ALI-FMM, arXiv 2302.10988).

Thin Python binding over the C ABI of libali.so (include/ali.h).  torch provides device
memory and the stream; every step of the computation runs in the HIP kernels.  There is
no CPU fallback: without the built library or a GPU, calls raise.
"""
from __future__ import annotations

import ctypes

from . import _lib

__all__ = ["AliError", "Batch", "Solver", "default_options"]

_MAT_FIELDS = ("c11", "c13", "c33", "c55", "c44", "c66", "rho")


class AliError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (status %d): %s" % (_status_string(status), status, message))
        self.status = status


def _status_string(status):
    try:
        return _lib.load().ali_status_string(status).decode()
    except Exception:  # library not loadable: still report the code
        return "status"


def default_options(_n_nodes=None, **overrides):
    lib = _lib.load()
    o = _lib.Options()
    lib.ali_default_options(ctypes.byref(o))
    for k, v in overrides.items():
        if v is not None:
            if k == "wave" and isinstance(v, str):
                v = _lib.WAVE[v]
            if k == "velocity" and isinstance(v, str):
                v = _lib.VELOCITY[v]
            if k == "node_A":
                # per-node A11, A13, A33, A55 [.., 4] float32 device tensor, in the node order
                # of the medium arrays (the caller keeps it alive for the call)
                import torch
                if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.float32
                        and v.is_contiguous() and v.dim() >= 2 and v.shape[-1] == 4):
                    raise ValueError("node_A must be a contiguous float32 device tensor [..., 4]")
                if _n_nodes is not None and v.numel() != 4 * _n_nodes:
                    raise ValueError("node_A needs 4 values per node (%d nodes)" % _n_nodes)
                o.d_node_A = v.data_ptr()
                continue
            setattr(o, k, int(v))
    return o


def _materials(mats):
    mats = list(mats)
    arr = (_lib.Material * len(mats))()
    for k, m in enumerate(mats):
        vals = [m[n] for n in _MAT_FIELDS] if isinstance(m, dict) else list(m)
        for n, v in zip(_MAT_FIELDS, vals):
            setattr(arr[k], n, float(v))
    return arr, len(mats)


def _nodes(nodes):
    nodes = [tuple(int(v) for v in p) for p in nodes]
    arr = (_lib.Node * max(len(nodes), 1))()
    for k, (i, j) in enumerate(nodes):
        arr[k].i, arr[k].j = i, j
    return arr, len(nodes)


def _refine(levels, start_half_width, subgrid):
    levels = [tuple(v) for v in levels]
    if len(levels) > _lib.MAX_LEVELS:
        raise ValueError("at most %d levels" % _lib.MAX_LEVELS)
    ref = _lib.Refine()
    ref.n_levels = len(levels)
    for k, (d, r) in enumerate(levels):
        ref.density[k] = int(d)
        ref.radius[k] = int(r)
    ref.start_half_width = float(start_half_width)
    ref.subgrid = int(subgrid)
    return ref


def _dev_ptr(t, dtype, shape=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must have dtype %s" % (name, dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


class Batch:
    """Media packed for the batch entry points: one material table, per-node arrays of all
    media concatenated on the device, sources and receivers concatenated on the host.

    media: sequence of objects with attributes nx, nz, h, mats, mat_id [nz, nx] (uint8
    array), orient [nz, nx] (radians), sources [(i, j)], receivers [(i, j)]."""

    def __init__(self, media, device="cuda"):
        import numpy as np
        import torch
        descs, mats, srcs, recs, ids, oris = [], [], [], [], [], []
        node = 0
        for m in media:
            d = _lib.Medium()
            d.grid = _lib.Grid(int(m.nx), int(m.nz), float(m.h))
            d.mat_offset, d.n_mats = len(mats), len(m.mats)
            d.node_offset = node
            d.src_offset, d.n_src = len(srcs), len(m.sources)
            d.rec_offset, d.n_rec = len(recs), len(getattr(m, "receivers", []) or [])
            mats.extend(m.mats)
            srcs.extend(m.sources)
            recs.extend(getattr(m, "receivers", []) or [])
            ids.append(np.ascontiguousarray(m.mat_id, dtype=np.uint8).ravel())
            oris.append(np.ascontiguousarray(m.orient, dtype=np.float32).ravel())
            node += int(m.nx) * int(m.nz)
            descs.append(d)
        self.n_media = len(descs)
        self.media = (_lib.Medium * self.n_media)(*descs)
        self.mats, self.n_mats = _materials(mats)
        self.srcs, self.n_src = _nodes(srcs)
        self.recs, self.n_rec = _nodes(recs) if recs else (None, 0)
        self.mat_id = torch.from_numpy(np.concatenate(ids)).to(device)
        self.orient = torch.from_numpy(np.concatenate(oris)).to(device)
        self.shapes = [(int(d.grid.nz), int(d.grid.nx)) for d in descs]
        self.n_fields = sum(int(d.n_src) for d in descs)
        self.field_nodes = sum(int(d.n_src) * int(d.grid.nx) * int(d.grid.nz) for d in descs)
        self.n_obs = sum(int(d.n_src) * int(d.n_rec) for d in descs)

    def fields(self, T):
        """Split a batch output [field_nodes] into per-medium [n_src, nz, nx] views."""
        out, off = [], 0
        for d, (nz, nx) in zip(self.media, self.shapes):
            n = int(d.n_src) * nz * nx
            out.append(T[off:off + n].view(int(d.n_src), nz, nx))
            off += n
        return out

    def per_node(self, a):
        """Split a per-node array (orientation layout) into per-medium [nz, nx] views."""
        out = []
        for d, (nz, nx) in zip(self.media, self.shapes):
            off = int(d.node_offset)
            out.append(a[off:off + nz * nx].view(nz, nx))
        return out


class Solver:
    """One handle of the C ABI, bound to a device and to torch's current stream."""

    def __init__(self, device=None):
        import torch
        self._lib = _lib.load()
        dev = torch.cuda.current_device() if device is None else int(device)
        self.device = dev
        h = ctypes.c_void_p()
        stream = torch.cuda.current_stream(dev).cuda_stream
        st = self._lib.ali_create(ctypes.byref(h), dev, ctypes.c_void_p(stream))
        if st != 0:
            raise AliError(st, "ali_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.ali_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_barrier_timeout(self, seconds):
        """Wait limit of the persistent relaxation's grid barriers (default 5 s)."""
        self._check(self._lib.ali_set_barrier_timeout(self._h, float(seconds)))

    def _sync_stream(self):
        import torch
        self._lib.ali_set_stream(self._h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def _check(self, st):
        if st != 0:
            raise AliError(st, self._lib.ali_last_error(self._h).decode())

    def solve(self, h, mats, mat_id, orient, sources, out=None, precision="f32",
              src_box_radius=None, max_sweeps=None, inner_sweeps=None, band_cells=None,
              arith="mixed", noalloc=False, **extra):
        """Travel-time fields [n_src, nz, nx] for point sources in one medium.

        h: grid spacing [m]; mats: list of stiffness records (dicts with c11, c13, c33,
        c55, c44, c66 [Pa], rho [kg/m^3]); mat_id: uint8 [nz, nx] device tensor;
        orient: symmetry-axis angle [rad], float32 (float64 for precision="f64") [nz, nx];
        sources: [(i, j), ...]; arith (float32 output only): "mixed" (float64 times and
        decisions, float32 wavefront math), "f32" or "f64"; extra: other ali_options fields by
        name (wave="sh" for the shear wave polarised normal to the plane, velocity="table" for
        the paper's velocity table; node_A=[nz, nx, 4] float32 device tensor of every node's
        A11, A13, A33, A55 = C / rho in place of the material table, also taken by adjoint,
        misfit_gradient and the batch calls); noalloc=True (float32 only) calls the
        allocation-free entry point, whose scratch is a static device array (pass `out`
        to allocate nothing at all).  Returns (T, stats dict)."""
        import torch
        nz, nx = mat_id.shape
        fdt = torch.float32 if precision == "f32" else torch.float64
        m_arr, nm = _materials(mats)
        s_arr, ns = _nodes(sources)
        g = _lib.Grid(int(nx), int(nz), float(h))
        opt = default_options(src_box_radius=src_box_radius, max_sweeps=max_sweeps,
                              inner_sweeps=inner_sweeps, band_cells=band_cells,
                              arith=_lib.ARITH[arith], _n_nodes=int(nx) * int(nz), **extra)
        if out is None:
            out = torch.empty((ns, nz, nx), dtype=fdt, device=mat_id.device)
        p_id = _dev_ptr(mat_id, torch.uint8, (nz, nx), "mat_id")
        p_or = _dev_ptr(orient, fdt, (nz, nx), "orient")
        p_T = _dev_ptr(out, fdt, (ns, nz, nx), "out")
        stats = _lib.SolveStats()
        self._sync_stream()
        if noalloc and precision != "f32":
            raise ValueError("the allocation-free entry point is float32 only")
        fn = (self._lib.ali_solve_traveltime_noalloc if noalloc else self._lib.ali_solve_traveltime) \
            if precision == "f32" else self._lib.ali_solve_traveltime_f64
        st = fn(self._h, ctypes.byref(g), m_arr, nm, p_id, p_or, s_arr, ns, ctypes.byref(opt),
                p_T, ctypes.byref(stats))
        self._check(st)
        return out, stats.as_dict()

    def solve_refined(self, h, mats, mat_id, orient, sources, levels=None, start_half_width=None,
                      out=None, precision="f32", max_sweeps=None, inner_sweeps=None, band_cells=None,
                      arith="mixed", subgrid=1, **extra):
        """Travel-time fields [n_src, nz, nx] with nested fine grids around every source
        (Section 4.4): levels = ((density, radius), ...) from the finest; straight rays on the
        finest grid within start_half_width cells of the source.  subgrid = s (odd) solves on
        the s-fold refined medium and returns its fields at the given nodes (Section 4.5);
        levels and start_half_width then count cells of that grid.  By default the paper's
        choices: ((27, 1), (9, 6), (3, 13)) and 0.5 without a subgrid, ((9, 2 s), (3, 5 s))
        and s / 2 with one (Table 3).  Other arguments as solve.  Returns (T, stats dict)."""
        import torch
        s = int(subgrid)
        if levels is None:
            levels = ((27, 1), (9, 6), (3, 13)) if s <= 1 else ((9, 2 * s), (3, 5 * s))
        if start_half_width is None:
            start_half_width = 0.5 * max(s, 1)
        nz, nx = mat_id.shape
        fdt = torch.float32 if precision == "f32" else torch.float64
        m_arr, nm = _materials(mats)
        s_arr, ns = _nodes(sources)
        g = _lib.Grid(int(nx), int(nz), float(h))
        opt = default_options(max_sweeps=max_sweeps, inner_sweeps=inner_sweeps, band_cells=band_cells,
                              arith=_lib.ARITH[arith], _n_nodes=int(nx) * int(nz), **extra)
        ref = _refine(levels, start_half_width, s)
        if out is None:
            out = torch.empty((ns, nz, nx), dtype=fdt, device=mat_id.device)
        p_id = _dev_ptr(mat_id, torch.uint8, (nz, nx), "mat_id")
        p_or = _dev_ptr(orient, fdt, (nz, nx), "orient")
        p_T = _dev_ptr(out, fdt, (ns, nz, nx), "out")
        stats = _lib.SolveStats()
        self._sync_stream()
        fn = (self._lib.ali_solve_traveltime_refined if precision == "f32"
              else self._lib.ali_solve_traveltime_refined_f64)
        st = fn(self._h, ctypes.byref(g), m_arr, nm, p_id, p_or, s_arr, ns, ctypes.byref(opt), ctypes.byref(ref),
                p_T, ctypes.byref(stats))
        self._check(st)
        return out, stats.as_dict()

    def trace_rays(self, h, mats, mat_id, orient, T, sources, receivers, window=None, sub=None,
                   max_pts=None, wave=None, planes=None, velocity=None, **extra):
        """Ray paths from every receiver to every source through the fields T
        [n_src, nz, nx] (float32 or float64 device tensor); wave "qp" (default) or "sh" as
        for the fields; planes "changing" (default), "x", "z", "diag", "anti" (one fixed
        family) or "fastest" (the fastest of the four fixed families); velocity
        "christoffel" (default) or "table" as for the fields.  Returns (paths [n_src, n_rec, max_pts, 2] float32 grid coordinates,
        npts [n_src, n_rec] int32 (negative: source not reached), tray [n_src, n_rec]
        float32 seconds)."""
        import torch
        nz, nx = mat_id.shape
        m_arr, nm = _materials(mats)
        s_arr, ns = _nodes(sources)
        r_arr, nr = _nodes(receivers)
        g = _lib.Grid(int(nx), int(nz), float(h))
        opt = default_options(ray_window=window, ray_sub=sub, ray_max_pts=max_pts, wave=wave, velocity=velocity,
                              ray_planes=_lib.RAY_PLANES[planes] if planes is not None else None, **extra)
        dev = mat_id.device
        paths = torch.empty((ns, nr, opt.ray_max_pts, 2), dtype=torch.float32, device=dev)
        npts = torch.empty((ns, nr), dtype=torch.int32, device=dev)
        tray = torch.empty((ns, nr), dtype=torch.float32, device=dev)
        p_id = _dev_ptr(mat_id, torch.uint8, (nz, nx), "mat_id")
        p_or = _dev_ptr(orient, torch.float32, (nz, nx), "orient")
        if T.dtype == torch.float64:
            fn, tdt = self._lib.ali_trace_rays_f64, torch.float64
        else:
            fn, tdt = self._lib.ali_trace_rays, torch.float32
        p_T = _dev_ptr(T, tdt, (ns, nz, nx), "T")
        self._sync_stream()
        st = fn(self._h, ctypes.byref(g), m_arr, nm, p_id, p_or, p_T, s_arr, ns, r_arr, nr,
                ctypes.byref(opt), _dev_ptr(paths, torch.float32), _dev_ptr(npts, torch.int32),
                _dev_ptr(tray, torch.float32))
        self._check(st)
        return paths, npts, tray

    def adjoint(self, h, mats, mat_id, orient, sources, receivers, dLdT, precision="f32",
                return_T=False, src_box_radius=None, max_sweeps=None, inner_sweeps=None,
                band_cells=None, arith="mixed", stiffness=False, **extra):
        """dL/dtheta [nz, nx] (summed over sources) for dL/dT given at the receivers,
        dLdT [n_src, n_rec] device tensor.  The forward fields are solved inside the call
        (returned when return_T).  precision "f32" (arith "mixed" or "f64") or "f64".
        stiffness=True also returns dL/dA [nz, nx, 4] (A11, A13, A33, A55 of every node,
        A = C / rho), as a tuple (dLdtheta, dLdA) in place of dLdtheta.
        Returns (dLdtheta, stats dict) or (dLdtheta, T, stats dict)."""
        import torch
        nz, nx = mat_id.shape
        fdt = torch.float32 if precision == "f32" else torch.float64
        m_arr, nm = _materials(mats)
        s_arr, ns = _nodes(sources)
        r_arr, nr = _nodes(receivers)
        g = _lib.Grid(int(nx), int(nz), float(h))
        opt = default_options(src_box_radius=src_box_radius, max_sweeps=max_sweeps,
                              inner_sweeps=inner_sweeps, band_cells=band_cells,
                              arith=_lib.ARITH[arith], _n_nodes=int(nx) * int(nz), **extra)
        dev = mat_id.device
        dth = torch.empty((nz, nx), dtype=fdt, device=dev)
        T = torch.empty((ns, nz, nx), dtype=fdt, device=dev) if return_T else None
        stats = _lib.AdjointStats()
        self._sync_stream()
        args = [self._h, ctypes.byref(g), m_arr, nm, _dev_ptr(mat_id, torch.uint8, (nz, nx), "mat_id"),
                _dev_ptr(orient, fdt, (nz, nx), "orient"), s_arr, ns, r_arr, nr,
                _dev_ptr(dLdT, fdt, (ns, nr), "dLdT"), ctypes.byref(opt),
                _dev_ptr(T, fdt) if T is not None else None, _dev_ptr(dth, fdt)]
        if stiffness:
            dA = torch.empty((nz, nx, 4), dtype=fdt, device=dev)
            fn = self._lib.ali_adjoint_stiffness if precision == "f32" else self._lib.ali_adjoint_stiffness_f64
            st = fn(*args, _dev_ptr(dA, fdt), ctypes.byref(stats))
            grad = (dth, dA)
        else:
            fn = self._lib.ali_adjoint if precision == "f32" else self._lib.ali_adjoint_f64
            st = fn(*args, ctypes.byref(stats))
            grad = dth
        self._check(st)
        return (grad, T, stats.as_dict()) if return_T else (grad, stats.as_dict())

    def misfit_gradient(self, h, mats, mat_id, orient, sources, receivers, obs, precision="f32",
                        T_out=None, src_box_radius=None, max_sweeps=None, inner_sweeps=None,
                        band_cells=None, arith="mixed", stiffness=False, subgrid=1, **extra):
        """Forward + adjoint of L = 1/2 sum (T_s(r) - obs[s, r])^2 in one call; the forward
        fields go to T_out [n_src, nz, nx] when given.  stiffness=True returns (dLdtheta,
        dLdA [nz, nx, 4]) in place of dLdtheta (as adjoint).  subgrid = s (odd) runs the
        forward and adjoint on the medium refined s-fold and sums the gradient back onto the
        nodes (ali_misfit_gradient_subgrid; orientation only).
        Returns (loss float64 device scalar, Trec [n_src, n_rec], dLdtheta [nz, nx], stats)."""
        import torch
        nz, nx = mat_id.shape
        fdt = torch.float32 if precision == "f32" else torch.float64
        m_arr, nm = _materials(mats)
        s_arr, ns = _nodes(sources)
        r_arr, nr = _nodes(receivers)
        g = _lib.Grid(int(nx), int(nz), float(h))
        opt = default_options(src_box_radius=src_box_radius, max_sweeps=max_sweeps,
                              inner_sweeps=inner_sweeps, band_cells=band_cells,
                              arith=_lib.ARITH[arith], _n_nodes=int(nx) * int(nz), **extra)
        dev = mat_id.device
        dth = torch.empty((nz, nx), dtype=fdt, device=dev)
        trec = torch.empty((ns, nr), dtype=fdt, device=dev)
        loss = torch.empty((), dtype=torch.float64, device=dev)
        stats = _lib.AdjointStats()
        self._sync_stream()
        args = [self._h, ctypes.byref(g), m_arr, nm, _dev_ptr(mat_id, torch.uint8, (nz, nx), "mat_id"),
                _dev_ptr(orient, fdt, (nz, nx), "orient"), s_arr, ns, r_arr, nr,
                _dev_ptr(obs, fdt, (ns, nr), "obs"), ctypes.byref(opt),
                _dev_ptr(T_out, fdt, (ns, nz, nx), "T_out") if T_out is not None else None, _dev_ptr(trec, fdt),
                _dev_ptr(loss, torch.float64), _dev_ptr(dth, fdt)]
        if subgrid != 1:
            if stiffness:
                raise ValueError("the subgrid misfit gradient differentiates orientation only")
            fn = (self._lib.ali_misfit_gradient_subgrid if precision == "f32"
                  else self._lib.ali_misfit_gradient_subgrid_f64)
            st = fn(*args[:12], int(subgrid), *args[12:], ctypes.byref(stats))
            self._check(st)
            return loss, trec, dth, stats.as_dict()
        if stiffness:
            dA = torch.empty((nz, nx, 4), dtype=fdt, device=dev)
            fn = (self._lib.ali_misfit_gradient_stiffness if precision == "f32"
                  else self._lib.ali_misfit_gradient_stiffness_f64)
            st = fn(*args, _dev_ptr(dA, fdt), ctypes.byref(stats))
            grad = (dth, dA)
        else:
            fn = self._lib.ali_misfit_gradient if precision == "f32" else self._lib.ali_misfit_gradient_f64
            st = fn(*args, ctypes.byref(stats))
            grad = dth
        self._check(st)
        return loss, trec, grad, stats.as_dict()

    def bilinear(self, ctrl, nz, nx):
        """Orientation [nz, nx] from control values ctrl [ncz, ncx] (float32 or float64
        device tensor) spanning the grid corner to corner, linear in each direction."""
        import torch
        ncz, ncx = ctrl.shape
        out = torch.empty((nz, nx), dtype=ctrl.dtype, device=ctrl.device)
        fn = self._lib.ali_bilinear if ctrl.dtype == torch.float32 else self._lib.ali_bilinear_f64
        self._sync_stream()
        self._check(fn(self._h, int(nz), int(nx), int(ncz), int(ncx), _dev_ptr(ctrl, ctrl.dtype, name="ctrl"),
                       _dev_ptr(out, ctrl.dtype)))
        return out

    def bilinear_transpose(self, g, ncz, ncx):
        """Transpose of bilinear: dL/dcontrol [ncz, ncx] from dL/dtheta [nz, nx]."""
        import torch
        nz, nx = g.shape
        out = torch.empty((ncz, ncx), dtype=g.dtype, device=g.device)
        fn = self._lib.ali_bilinear_transpose if g.dtype == torch.float32 else self._lib.ali_bilinear_transpose_f64
        self._sync_stream()
        self._check(fn(self._h, int(nz), int(nx), int(ncz), int(ncx), _dev_ptr(g, g.dtype, name="dLdtheta"),
                       _dev_ptr(out, g.dtype)))
        return out


    def solve_batch(self, batch, out=None, arith="mixed", **opts):
        """Fields of every source of every medium of `batch` in one call.  Returns (T
        [field_nodes] float32 in medium order, stats dict)."""
        import torch
        opt = default_options(arith=_lib.ARITH[arith], _n_nodes=batch.mat_id.numel(), **opts)
        if out is None:
            out = torch.empty(batch.field_nodes, dtype=torch.float32, device=batch.mat_id.device)
        stats = _lib.SolveStats()
        self._sync_stream()
        st = self._lib.ali_solve_batch(self._h, batch.media, batch.n_media, batch.mats, batch.n_mats,
                                       _dev_ptr(batch.mat_id, torch.uint8, name="mat_id"),
                                       _dev_ptr(batch.orient, torch.float32, name="orient"), batch.srcs,
                                       ctypes.byref(opt), _dev_ptr(out, torch.float32, (batch.field_nodes,), "out"),
                                       ctypes.byref(stats))
        self._check(st)
        return out, stats.as_dict()

    def solve_batch_refined(self, batch, levels=None, start_half_width=0.5, out=None, arith="mixed", **opts):
        """solve_batch with nested fine grids around every source of every medium (Section
        4.4), levels and start_half_width as in solve_refined (default: the paper's
        ((27, 1), (9, 6), (3, 13)) and 0.5).  Returns (T [field_nodes] float32 in medium
        order, stats dict)."""
        import torch
        if levels is None:
            levels = ((27, 1), (9, 6), (3, 13))
        ref = _refine(levels, start_half_width, 1)
        opt = default_options(arith=_lib.ARITH[arith], _n_nodes=batch.mat_id.numel(), **opts)
        if out is None:
            out = torch.empty(batch.field_nodes, dtype=torch.float32, device=batch.mat_id.device)
        stats = _lib.SolveStats()
        self._sync_stream()
        st = self._lib.ali_solve_batch_refined(self._h, batch.media, batch.n_media, batch.mats, batch.n_mats,
                                               _dev_ptr(batch.mat_id, torch.uint8, name="mat_id"),
                                               _dev_ptr(batch.orient, torch.float32, name="orient"), batch.srcs,
                                               ctypes.byref(opt), ctypes.byref(ref),
                                               _dev_ptr(out, torch.float32, (batch.field_nodes,), "out"),
                                               ctypes.byref(stats))
        self._check(st)
        return out, stats.as_dict()

    def misfit_gradient_batch(self, batch, obs, orient=None, arith="mixed", stiffness=False, **opts):
        """Forward + adjoint of the receiver misfit for every medium of `batch` in one call.
        obs: [n_obs] float32 device tensor (per field, its medium's receivers); orient: optional
        replacement of the batch's orientation (same layout).  stiffness=True returns
        (dLdtheta, dLdA [nodes, 4]) in place of dLdtheta.  Returns (loss [n_media] float64,
        Trec [n_obs], dLdtheta [nodes] float32, stats)."""
        import torch
        opt = default_options(arith=_lib.ARITH[arith], _n_nodes=batch.mat_id.numel(), **opts)
        dev = batch.mat_id.device
        ori = batch.orient if orient is None else orient
        dth = torch.empty_like(batch.orient)
        trec = torch.empty(batch.n_obs, dtype=torch.float32, device=dev)
        loss = torch.empty(batch.n_media, dtype=torch.float64, device=dev)
        stats = _lib.AdjointStats()
        self._sync_stream()
        args = [self._h, batch.media, batch.n_media, batch.mats, batch.n_mats,
                _dev_ptr(batch.mat_id, torch.uint8, name="mat_id"),
                _dev_ptr(ori, torch.float32, tuple(batch.orient.shape), "orient"),
                batch.srcs, batch.recs, _dev_ptr(obs, torch.float32, (batch.n_obs,), "obs"),
                ctypes.byref(opt), _dev_ptr(trec, torch.float32),
                _dev_ptr(loss, torch.float64), _dev_ptr(dth, torch.float32)]
        if stiffness:
            dA = torch.empty(tuple(batch.orient.shape) + (4,), dtype=torch.float32, device=dev)
            st = self._lib.ali_misfit_gradient_batch_stiffness(*args, _dev_ptr(dA, torch.float32), ctypes.byref(stats))
            grad = (dth, dA)
        else:
            st = self._lib.ali_misfit_gradient_batch(*args, ctypes.byref(stats))
            grad = dth
        self._check(st)
        return loss, trec, grad, stats.as_dict()

    def autotune_batch(self, batch, arith="mixed", cache_file=None, **opts):
        """Time the forward batch solve under each candidate schedule and return (the
        fastest options as a dict, {(band_cells, inner_sweeps, visit_tiles, persistent): ms},
        cached).  The handle
        keeps the choice per size bucket (a second call with a batch of the same bucket
        times nothing); cache_file (JSON, optional) keeps it across processes under the
        same bucket key.  cached is True when no candidate was timed."""
        import json
        import os
        import torch
        opt = default_options(arith=_lib.ARITH[arith], _n_nodes=batch.mat_id.numel(), **opts)
        key = tune_bucket(batch, opt)
        if cache_file and os.path.exists(cache_file):
            with open(cache_file) as fh:
                hit = json.load(fh).get(key)
            if hit is not None:
                for k, v in hit["choice"].items():
                    setattr(opt, k, int(v))
                best = {k: getattr(opt, k) for k, _ in opt._fields_}
                return best, {tuple(c): ms for c, ms in hit["ms"]}, True
        out = torch.empty(batch.field_nodes, dtype=torch.float32, device=batch.mat_id.device)
        ms = (ctypes.c_double * len(_lib.TUNE_CANDIDATES))()
        self._sync_stream()
        st = self._lib.ali_autotune_batch(self._h, batch.media, batch.n_media, batch.mats, batch.n_mats,
                                          _dev_ptr(batch.mat_id, torch.uint8, name="mat_id"),
                                          _dev_ptr(batch.orient, torch.float32, name="orient"), batch.srcs,
                                          ctypes.byref(opt), _dev_ptr(out, torch.float32), ms)
        self._check(st)
        best = {k: getattr(opt, k) for k, _ in opt._fields_}
        times = {c: ms[k] for k, c in enumerate(_lib.TUNE_CANDIDATES)}
        if cache_file:
            data = {}
            if os.path.exists(cache_file):
                with open(cache_file) as fh:
                    data = json.load(fh)
            data[key] = {"choice": {k: best[k] for k in _lib.TUNE_KNOBS},
                         "ms": [[list(c), v] for c, v in times.items()]}
            tmp = cache_file + ".tmp%d" % os.getpid()
            with open(tmp, "w") as fh:
                json.dump(data, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache_file)
        return best, times, False


def tune_bucket(batch, opt):
    """Size bucket of a batch for the schedule cache: powers of two of the field count, the
    largest side and the node-fields, with the arithmetic, wave and speed mode."""
    def p2(v):
        return max(int(v) - 1, 0).bit_length()
    side = max(max(nz, nx) for nz, nx in batch.shapes)
    return "v%d:f%d:s%d:n%d:a%d:w%d:v%d:A%d" % (_lib.TUNE_VERSION, p2(batch.n_fields), p2(side),
                                               p2(batch.field_nodes), opt.arith, opt.wave, opt.velocity,
                                               1 if opt.d_node_A else 0)


def receiver_times(solver, h, mats, mat_id, orient, sources, receivers, node_A=None, **opts):
    """Travel times [n_src, n_rec] at the receivers as a differentiable function of the
    orientation [nz, nx] (float32 device tensor; float64 solves in float64 throughout) and,
    when given, of the per-node stiffness node_A [nz, nx, 4] (float32 device tensor of
    A11, A13, A33, A55 = C / rho of every node, in place of the material table).  The
    backward pass runs the adjoint kernels (the forward fields are solved again inside it,
    not stored) and returns dL/dtheta and, when node_A requires a gradient, dL/dA."""
    return _ReceiverTimes.apply(orient, node_A, solver, h, mats, mat_id, tuple(map(tuple, sources)),
                                tuple(map(tuple, receivers)), opts)


def bilinear_orientation(solver, ctrl, nz, nx):
    """Orientation [nz, nx] from control values ctrl [ncz, ncx] spanning the grid corner to
    corner (linear in each direction), differentiable in ctrl (backward: the transpose)."""
    return _Bilinear.apply(ctrl, solver, int(nz), int(nx))


def _autograd():
    import torch

    class ReceiverTimes(torch.autograd.Function):
        @staticmethod
        def forward(ctx, orient, node_A, solver, h, mats, mat_id, sources, receivers, opts):
            prec = "f64" if orient.dtype == torch.float64 else "f32"
            kw = dict(opts)
            if node_A is not None:
                kw["node_A"] = node_A.detach()
            T, _ = solver.solve(h, mats, mat_id, orient.detach(), sources, precision=prec, **kw)
            rows = torch.tensor([r[1] for r in receivers], device=T.device)
            cols = torch.tensor([r[0] for r in receivers], device=T.device)
            ctx.save_for_backward(orient, node_A)
            ctx.args = (solver, h, mats, mat_id, sources, receivers, kw, prec)
            return T[:, rows, cols].contiguous()

        @staticmethod
        def backward(ctx, grad):
            orient, node_A = ctx.saved_tensors
            solver, h, mats, mat_id, sources, receivers, kw, prec = ctx.args
            want_A = node_A is not None and ctx.needs_input_grad[1]
            g = grad.to(orient.dtype).contiguous()
            res, _ = solver.adjoint(h, mats, mat_id, orient.detach(), sources, receivers, g, precision=prec,
                                    stiffness=want_A, **kw)
            if want_A:
                dth, dA = res
                dA = dA.to(node_A.dtype).view(node_A.shape)
            else:
                dth, dA = res, None
            return dth, dA, None, None, None, None, None, None, None

    class Bilinear(torch.autograd.Function):
        @staticmethod
        def forward(ctx, ctrl, solver, nz, nx):
            ctx.args = (solver, ctrl.shape[0], ctrl.shape[1])
            return solver.bilinear(ctrl.contiguous(), nz, nx)

        @staticmethod
        def backward(ctx, grad):
            solver, ncz, ncx = ctx.args
            return solver.bilinear_transpose(grad.contiguous(), ncz, ncx), None, None, None

    return ReceiverTimes, Bilinear


class _Lazy:
    """Defer importing torch until a differentiable function is first used."""

    def __init__(self, k):
        self.k = k

    def apply(self, *a):
        return _autograd()[self.k].apply(*a)


_ReceiverTimes, _Bilinear = _Lazy(0), _Lazy(1)
__all__ += ["receiver_times", "bilinear_orientation"]
