"""Python binding of libcm (argument marshalling only).

PyTorch supplies device memory and streams; every step of the contact-manifold
path runs in the HIP kernels behind the C ABI (include/cm.h).  There is no CPU
fallback: if libcm.so or a HIP device is missing, these calls raise.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib as L


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _np_ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _stream_handle(stream: Optional[torch.cuda.Stream]):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


@dataclass
class DeviceBatch:
    """A scene batch resident on the device (int32 / float32 tensors)."""
    n_scenes: int
    n_bodies: int
    body_offsets: torch.Tensor
    body_geom: torch.Tensor
    pose: torch.Tensor
    cand_offsets: Optional[torch.Tensor] = None
    cand_pairs: Optional[torch.Tensor] = None

    @property
    def n_cand_total(self) -> int:
        if self.cand_pairs is not None:
            return int(self.cand_pairs.shape[1])
        bo = self.body_offsets.cpu().numpy().astype(np.int64)
        nb = np.diff(bo)
        return int((nb * (nb - 1) // 2).sum())

    def validate(self):
        """Check dtypes, shapes and placement before the pointers cross the C ABI."""
        def need(t, name, dtype, shape):
            if not isinstance(t, torch.Tensor):
                raise TypeError(f"{name} must be a torch tensor")
            if t.dtype != dtype:
                raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
            if tuple(t.shape) != shape:
                raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous device tensor")
        need(self.body_offsets, "body_offsets", torch.int32, (self.n_scenes + 1,))
        need(self.body_geom, "body_geom", torch.int32, (self.n_bodies,))
        need(self.pose, "pose", torch.float32, (7, self.n_bodies))
        if (self.cand_offsets is None) != (self.cand_pairs is None):
            raise ValueError("cand_offsets and cand_pairs go together")
        if self.cand_pairs is not None:
            need(self.cand_offsets, "cand_offsets", torch.int32, (self.n_scenes + 1,))
            need(self.cand_pairs, "cand_pairs", torch.int32, (2, int(self.cand_pairs.shape[1])))

    def as_c(self) -> L.cm_batch:
        self.validate()
        b = L.cm_batch()
        b.n_scenes = self.n_scenes
        b.n_bodies = self.n_bodies
        b.body_offsets = _ptr(self.body_offsets)
        b.body_geom = _ptr(self.body_geom)
        b.pose = _ptr(self.pose)
        b.cand_offsets = _ptr(self.cand_offsets)
        b.cand_pairs = _ptr(self.cand_pairs)
        b.n_cand = 0 if self.cand_pairs is None else int(self.cand_pairs.shape[1])
        return b


@dataclass
class Manifold:
    """Caller-owned manifold outputs (device tensors)."""
    K: int
    capacity: int
    n_pairs: torch.Tensor       # int32 [1]
    pair_offsets: torch.Tensor  # int32 [S+1]
    pairs: torch.Tensor         # int32 [2, cap]
    point: torch.Tensor         # float32 [3, cap*K]
    normal: torch.Tensor        # float32 [3, cap*K]
    dist: torch.Tensor          # float32 [cap*K]
    weight: torch.Tensor        # float32 [cap*K]
    tape: Optional[torch.Tensor] = None   # uint8 [cm_tape_bytes]: the adjoint's tape, when recorded

    @staticmethod
    def empty(n_scenes: int, capacity: int, K: int, device) -> "Manifold":
        z32 = lambda *s: torch.zeros(*s, dtype=torch.int32, device=device)
        f32 = lambda *s: torch.zeros(*s, dtype=torch.float32, device=device)
        cap = max(int(capacity), 0)
        return Manifold(K, cap, z32(1), z32(n_scenes + 1), z32(2, max(cap, 1)), f32(3, max(cap * K, 1)),
                        f32(3, max(cap * K, 1)), f32(max(cap * K, 1)), f32(max(cap * K, 1)))

    def as_c(self) -> L.cm_manifold:
        m = L.cm_manifold()
        m.capacity = self.capacity
        m.n_pairs = _ptr(self.n_pairs)
        m.pair_offsets = _ptr(self.pair_offsets)
        m.pairs = _ptr(self.pairs)
        m.point = _ptr(self.point)
        m.normal = _ptr(self.normal)
        m.dist = _ptr(self.dist)
        m.weight = _ptr(self.weight)
        m.tape = _ptr(self.tape) if self.tape is not None else None
        m.tape_bytes = int(self.tape.numel()) if self.tape is not None else 0
        return m

    def to_numpy(self):
        """Host copy: pairs [2,n], offsets, p [n,K,3], nu [n,K,3], d [n,K], w [n,K]."""
        n = min(int(self.n_pairs.item()), self.capacity)
        K = self.K
        p = self.point[:, :n * K].cpu().numpy().reshape(3, n, K).transpose(1, 2, 0)
        nu = self.normal[:, :n * K].cpu().numpy().reshape(3, n, K).transpose(1, 2, 0)
        return dict(n_pairs=int(self.n_pairs.item()), pairs=self.pairs[:, :n].cpu().numpy(),
                    offsets=self.pair_offsets.cpu().numpy(), p=p, nu=nu,
                    d=self.dist[:n * K].cpu().numpy().reshape(n, K), w=self.weight[:n * K].cpu().numpy().reshape(n, K))


FLAG_NO_EE = 1          # no edge-edge candidates
FLAG_ONE_SIDED_VS = 2   # vertex-SDF candidates of the first body only
FLAG_SAFEGUARD = 4      # with pre-selection: scale E-E activities by the inside indicators


def make_params(tau: float, K: int, lambda_reg: float = -1.0, eps_n: float = -1.0, cull_margin: float = -1.0,
                flags: int = 0, presel=None, refine: int = 0):
    """presel: None, or (K_V, K_E) for soft top-K pre-selection; refine:
    sphere-tracing steps of the E-E witnesses (0 = off)."""
    p = L.cm_params()
    p.tau, p.K, p.lambda_reg, p.eps_n, p.cull_margin = float(tau), int(K), lambda_reg, eps_n, cull_margin
    p.flags = int(flags)
    p.presel_vertices, p.presel_edges = (0, 0) if presel is None else (int(presel[0]), int(presel[1]))
    p.refine_steps = int(refine)
    return p


class Context:
    """A libcm context on one HIP device (owns geometry tables and workspace)."""

    def __init__(self, device: int = 0):
        self.lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("libcm needs a HIP device (no CPU fallback)")
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        self._check(self.lib.cm_context_create(device, C.byref(h)), ctx=None)
        self.h = h

    def _check(self, status, ctx="self"):
        if status != L.CM_OK:
            msg = ""
            if ctx is not None and getattr(self, "h", None):
                msg = self.lib.cm_last_error(self.h).decode()
            raise L.CMError(status, msg)

    def close(self):
        if getattr(self, "h", None):
            self.lib.cm_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- geometry
    def create_geometry(self, geoms) -> np.ndarray:
        """Create all geometries of a workloads.GeomSet; returns their ids."""
        n = geoms.n
        types = np.ascontiguousarray(geoms.types, dtype=np.int32)
        params = np.ascontiguousarray(geoms.params, dtype=np.float32)
        off = np.ascontiguousarray(geoms.pt_off, dtype=np.int64)
        pts = np.ascontiguousarray(geoms.points, dtype=np.float32).reshape(-1)
        if pts.size == 0:
            pts = np.zeros(3, np.float32)
        ids = np.zeros(n, dtype=np.int32)
        self._check(self.lib.cm_geometry_create(self.h, n, _np_ptr(types), _np_ptr(params), _np_ptr(off),
                                                _np_ptr(pts), _np_ptr(ids)))
        return ids

    def geometry_info(self, gid: int) -> dict:
        info = L.cm_geometry_info_t()
        self._check(self.lib.cm_geometry_info(self.h, int(gid), C.byref(info)))
        return dict(type=info.type, n_vertices=info.n_vertices, n_edges=info.n_edges, n_faces=info.n_faces,
                    vertex_offset=info.vertex_offset, bound_radius=info.bound_radius)

    def geometry_mesh(self, gid: int):
        info = self.geometry_info(gid)
        v = np.zeros(3 * info["n_vertices"], np.float32)
        e = np.zeros(2 * info["n_edges"], np.int32)
        f = np.zeros(max(3 * info["n_faces"], 1), np.int32)
        self._check(self.lib.cm_geometry_mesh(self.h, int(gid), _np_ptr(v), _np_ptr(e), _np_ptr(f)))
        return v.reshape(-1, 3), e.reshape(-1, 2), f[:3 * info["n_faces"]].reshape(-1, 3)

    def destroy_geometry(self, gids) -> None:
        """Destroy geometries (cm_geometry_destroy); ids stay reserved."""
        g = np.ascontiguousarray(np.atleast_1d(gids), dtype=np.int32)
        self._check(self.lib.cm_geometry_destroy(self.h, _np_ptr(g), int(g.size)))

    @property
    def vertex_pool_size(self) -> int:
        return int(self.lib.cm_vertex_pool_size(self.h))

    @property
    def geometry_count(self) -> int:
        return int(self.lib.cm_geometry_count(self.h))

    # ------------------------------------------------------------- batches
    def upload_batch(self, batch, geom_ids: np.ndarray) -> DeviceBatch:
        """Copy a workloads.Batch to the device, mapping its geometry ids."""
        dev = self.device
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(dev)
        db = DeviceBatch(batch.n_scenes, batch.n_bodies, t(batch.body_offsets, torch.int32),
                         t(geom_ids[batch.body_geom], torch.int32), t(batch.pose, torch.float32))
        if batch.cand_pairs is not None:
            db.cand_offsets = t(batch.cand_offsets, torch.int32)
            db.cand_pairs = t(batch.cand_pairs, torch.int32)
        return db

    def check_errors(self, stream=None):
        self._check(self.lib.cm_check_errors(self.h, _stream_handle(stream)))

    # -------------------------------------------------------------- timing
    def set_kernel_timing(self, enable: bool):
        """Record HIP events around every timed launch (resets the sums)."""
        self._check(self.lib.cm_set_kernel_timing(self.h, 1 if enable else 0))

    def kernel_time(self, timer: str):
        """(summed milliseconds, launches) of one timer since timing was enabled."""
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        self._check(self.lib.cm_kernel_time(self.h, L.TIMERS[timer], C.byref(ms), C.byref(n)))
        return ms.value, n.value

    # ------------------------------------------------------------- forward
    def collide(self, db: DeviceBatch, tau: float, K: int, capacity: Optional[int] = None, out: Manifold = None,
                fused: bool = False, stream=None, lambda_reg=-1.0, eps_n=-1.0, cull_margin=-1.0,
                flags: int = 0, presel=None, refine: int = 0, noalloc: bool = False,
                record: bool = False) -> Manifold:
        """fused: cm_collide_fused; noalloc: cm_collide_noalloc (workspace in
        the library's static device array; the caller allocates `out`);
        record: also record the adjoint's tape into out.tape (allocated here
        when missing or too small), which collide_backward then uses.  A
        forward without record leaves out.tape None."""
        if fused and noalloc:
            raise ValueError("fused and noalloc are different entry points")
        if out is None:
            cap = db.n_cand_total if capacity is None else capacity
            out = Manifold.empty(db.n_scenes, cap, K, self.device)
        if record:
            need = self.tape_bytes(out.capacity, K)
            if out.tape is None or out.tape.numel() < need:
                out.tape = torch.empty(need, dtype=torch.uint8, device=self.device)
        else:
            out.tape = None
        prm = make_params(tau, K, lambda_reg, eps_n, cull_margin, flags, presel, refine)
        b = db.as_c()
        m = out.as_c()
        fn = self.lib.cm_collide_fused if fused else (self.lib.cm_collide_noalloc if noalloc else self.lib.cm_collide)
        self._check(fn(self.h, C.byref(b), C.byref(prm), C.byref(m), _stream_handle(stream)))
        return out

    def fused_tuning(self) -> dict:
        """The fused path's per-size-class plan (cm_fused_tuning)."""
        a = [(C.c_int32 * 3)() for _ in range(4)]
        ms = (C.c_float * 9)()
        self._check(self.lib.cm_fused_tuning(self.h, a[0], a[1], a[2], ms, a[3]))
        return dict(class_max_edges=list(a[0]), class_blocks=list(a[1]), sample_pairs=list(a[2]),
                    sample_ms=[[ms[3 * c + j] for j in range(3)] for c in range(3)],
                    from_cache=[bool(x) for x in a[3]])

    def tape_bytes(self, capacity: int, K: int, pool_entries: int = 0) -> int:
        """Bytes of the adjoint's tape for `capacity` pairs at K (cm_tape_bytes)."""
        n = C.c_int64(0)
        self._check(self.lib.cm_tape_bytes(self.h, int(capacity), int(K), int(pool_entries), C.byref(n)))
        return int(n.value)

    # ------------------------------------------------------------- E-E witness points
    def ee_witness(self, edges: torch.Tensor, tau: float, lambda_reg: float = -1.0, hard: bool = False,
                   out: torch.Tensor = None, stream=None) -> torch.Tensor:
        """Witness points of independent edge pairs (cm_ee_witness).

        edges: float32 [12, n] on this device (rows a0, a1, b0, b1, xyz each);
        returns float32 [9, n]: alpha1, alpha2, con, e1 xyz, e2 xyz.
        """
        if edges.dtype != torch.float32 or edges.dim() != 2 or edges.shape[0] != 12 or not edges.is_contiguous():
            raise ValueError("edges must be a contiguous float32 [12, n] tensor")
        if edges.device != self.device:
            raise ValueError(f"edges must be on {self.device}")
        n = edges.shape[1]
        if out is None:
            out = torch.empty(9, n, dtype=torch.float32, device=self.device)
        elif out.dtype != torch.float32 or tuple(out.shape) != (9, n) or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 [9, n] tensor")
        self._check(self.lib.cm_ee_witness(self.h, _ptr(edges), n, float(tau), float(lambda_reg),
                                           1 if hard else 0, _ptr(out), _stream_handle(stream)))
        return out

    # ------------------------------------------------------------- backward
    def collide_backward(self, db: DeviceBatch, fwd: Manifold, tau: float, K: int, g_point=None, g_normal=None,
                         g_dist=None, g_weight=None, stream=None, want_vertices=True, want_params=True,
                         lambda_reg=-1.0, eps_n=-1.0, cull_margin=-1.0, flags: int = 0, presel=None,
                         refine: int = 0) -> dict:
        """Vector-Jacobian product of the manifold for the given cotangents.

        Returns device tensors: pose [6, n_bodies] (left twists rho, omega),
        vertices [3, vertex_pool] (polytope hull vertices), params
        [4, n_geometries] (analytic parameters), tau [1].
        """
        dev = self.device
        out = dict(pose=torch.empty(6, db.n_bodies, dtype=torch.float32, device=dev),
                   vertices=torch.empty(3, max(self.vertex_pool_size, 1), dtype=torch.float32, device=dev)
                   if want_vertices else None,
                   params=torch.empty(4, max(self.geometry_count, 1), dtype=torch.float32, device=dev)
                   if want_params else None,
                   tau=torch.empty(1, dtype=torch.float32, device=dev))
        cot = L.cm_cotangent()
        cot.g_point, cot.g_normal, cot.g_dist, cot.g_weight = (_ptr(t) for t in (g_point, g_normal, g_dist, g_weight))
        gr = L.cm_grads()
        gr.g_pose, gr.g_vertices, gr.g_params, gr.g_tau = (_ptr(out[k]) for k in ("pose", "vertices", "params", "tau"))
        prm = make_params(tau, K, lambda_reg, eps_n, cull_margin, flags, presel, refine)
        b = db.as_c()
        m = fwd.as_c()
        self._check(self.lib.cm_collide_backward(self.h, C.byref(b), C.byref(prm), C.byref(m), C.byref(cot),
                                                 C.byref(gr), _stream_handle(stream)))
        return out


class _CollideFn(torch.autograd.Function):
    """Differentiable manifold: inputs are zero-valued leaves standing for the
    pose twists, hull vertices, analytic parameters and tau; the forward runs
    cm_collide at the batch's poses, the backward cm_collide_backward."""

    @staticmethod
    def forward(fctx, xi, verts, params, tau_t, cmctx, db, K, capacity, fused, flags, presel, refine):
        tau = float(tau_t.item())
        m = cmctx.collide(db, tau, K, capacity, fused=fused, flags=flags, presel=presel, refine=refine, record=True)
        fctx.cm = (cmctx, db, m, tau, K, flags, presel, refine)
        fctx.mark_non_differentiable(m.n_pairs, m.pairs)
        return m.point, m.normal, m.dist, m.weight, m.n_pairs, m.pairs

    @staticmethod
    def backward(fctx, gp, gn, gd, gw, _n, _p):
        cmctx, db, m, tau, K, flags, presel, refine = fctx.cm
        c = lambda t: None if t is None else t.contiguous()
        g = cmctx.collide_backward(db, m, tau, K, c(gp), c(gn), c(gd), c(gw), flags=flags, presel=presel,
                                   refine=refine)
        return g["pose"], g["vertices"], g["params"], g["tau"], None, None, None, None, None, None, None, None


def collide_autograd(cmctx: Context, db: DeviceBatch, tau_t: torch.Tensor, K: int, xi=None, verts=None,
                     params=None, capacity=None, fused=False, flags: int = 0, presel=None, refine: int = 0):
    """Manifold outputs (point, normal, dist, weight, n_pairs, pairs) that
    autograd can differentiate.  ``xi`` [6, n_bodies] must be zeros (the
    twist at which the gradient is taken); ``verts`` [3, vertex_pool] and
    ``params`` [4, n_geometries] are placeholders that receive geometry
    gradients.  ``flags``, ``presel`` and ``refine`` select the
    simplifications, soft top-K pre-selection and witness sphere tracing for
    both passes."""
    dev = cmctx.device
    if xi is None:
        xi = torch.zeros(6, db.n_bodies, device=dev, requires_grad=True)
    if verts is None:
        verts = torch.zeros(3, max(cmctx.vertex_pool_size, 1), device=dev, requires_grad=True)
    if params is None:
        params = torch.zeros(4, max(cmctx.geometry_count, 1), device=dev, requires_grad=True)
    cap = db.n_cand_total if capacity is None else capacity
    return _CollideFn.apply(xi, verts, params, tau_t, cmctx, db, K, cap, fused, flags, presel, refine)


class Server:
    """Continuous-batching request loop over a context's resident geometry
    (cm_server_*).  Requests carry host arrays; results come back as numpy
    copies.  Thread-safe submit / poll."""

    def __init__(self, cmctx: Context, budget_bytes: int, n_streams: int = 4):
        self.ctx = cmctx
        self.lib = cmctx.lib
        h = C.c_void_p()
        self._check(self.lib.cm_server_create(cmctx.h, C.c_uint64(int(budget_bytes)), int(n_streams), C.byref(h)))
        self.h = h
        self._keep = {}

    def _check(self, status):
        if status != L.CM_OK:
            raise L.CMError(status, (self.lib.cm_server_last_error() or b"").decode())

    def set_host_budget(self, budget_bytes: int):
        """Pinned host bytes the unreleased results may hold (default 8 GiB)."""
        self._check(self.lib.cm_server_set_host_budget(self.h, C.c_uint64(int(budget_bytes))))

    def submit(self, body_offsets, body_geom, pose, tau: float, K: int, want_backward=False, cot_dist=None,
               cot_normal=None, capacity: int = 0, flags: int = 0, presel=None, refine: int = 0, cot_point=None,
               cot_weight=None, want_geometry=False) -> int:
        """body_geom are context geometry ids; pose float32 [7, n_bodies];
        cotangents host float32 arrays laid out like the outputs ([3, cap*K] /
        [cap*K]) or None (zero)."""
        bo = np.ascontiguousarray(body_offsets, np.int32)
        bg = np.ascontiguousarray(body_geom, np.int32)
        ps = np.ascontiguousarray(pose, np.float32)
        q = L.cm_request()
        q.n_scenes, q.n_bodies = len(bo) - 1, len(bg)
        q.body_offsets, q.body_geom, q.pose = _np_ptr(bo), _np_ptr(bg), _np_ptr(ps)
        q.params = make_params(tau, K, flags=flags, presel=presel, refine=refine)
        q.want_backward = int(bool(want_backward))
        cots = [None if c is None else np.ascontiguousarray(c, np.float32)
                for c in (cot_point, cot_normal, cot_dist, cot_weight)]
        q.cot_point, q.cot_normal, q.cot_dist, q.cot_weight = (_np_ptr(c) for c in cots)
        q.want_geometry_grads = int(bool(want_geometry))
        q.capacity = int(capacity)
        t = C.c_uint64()
        self._check(self.lib.cm_server_submit(self.h, C.byref(q), C.byref(t)))
        self._keep[t.value] = (K, q.n_scenes, q.n_bodies, bool(want_backward), bool(want_geometry and want_backward))
        return t.value

    def poll(self, ticket: int):
        """None while pending / running, else a dict of numpy results."""
        r = L.cm_result()
        st = self.lib.cm_server_poll(self.h, C.c_uint64(ticket), C.byref(r))
        if st == -4:
            return None
        if st == -6 and ticket not in self._keep:
            self._check(st)
        K, S, nb, bwd, geo = self._keep[ticket]
        out = dict(status=st, n_pairs=r.n_pairs, capacity=r.capacity, t_submit=r.t_submit, t_start=r.t_start,
                   t_done=r.t_done, footprint=r.footprint_bytes)
        if not r.point:
            return out
        n, cap = r.n_pairs, r.capacity
        m = min(n, cap)
        arr = lambda p, cnt: np.ctypeslib.as_array(p, shape=(cnt,)).copy()
        out["offsets"] = arr(r.pair_offsets, S + 1)
        pr = arr(r.pairs, 2 * max(cap, 1))
        out["pairs"] = np.stack([pr[:m], pr[cap:cap + m]])
        pt = arr(r.point, 3 * max(cap, 1) * K).reshape(3, -1)[:, :m * K]
        nv = arr(r.normal, 3 * max(cap, 1) * K).reshape(3, -1)[:, :m * K]
        out["p"] = pt.reshape(3, m, K).transpose(1, 2, 0)
        out["nu"] = nv.reshape(3, m, K).transpose(1, 2, 0)
        out["d"] = arr(r.dist, max(cap, 1) * K)[:m * K].reshape(m, K)
        out["w"] = arr(r.weight, max(cap, 1) * K)[:m * K].reshape(m, K)
        if bwd:
            out["g_pose"] = arr(r.g_pose, 6 * max(nb, 1)).reshape(6, -1)[:, :nb]
            out["g_tau"] = float(r.g_tau[0])
            if geo:
                out["g_vertices"] = arr(r.g_vertices, 3 * max(r.vertex_pool, 1)).reshape(3, -1)[:, :r.vertex_pool]
                out["g_params"] = arr(r.g_params, 4 * max(r.n_geometries, 1)).reshape(4, -1)[:, :r.n_geometries]
        return out

    def release(self, ticket: int):
        self.lib.cm_server_release(self.h, C.c_uint64(ticket))
        self._keep.pop(ticket, None)

    def stats(self):
        b = C.c_uint64()
        p = C.c_int32()
        r = C.c_int32()
        self.lib.cm_server_stats(self.h, C.byref(b), C.byref(p), C.byref(r))
        return dict(in_flight_bytes=b.value, pending=p.value, running=r.value)

    def close(self):
        if getattr(self, "h", None):
            self.lib.cm_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
