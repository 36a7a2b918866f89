"""Python binding of libpcrt, the MI355X point-cloud radio ray tracer.

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI declared in include/pcrt.h. PyTorch supplies device memory
and the stream. If the built library is missing, importing the binding
raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcrt.so")
LIB_COUNT_PATH = os.path.join(_HERE, "libpcrt_count.so")  # measurement build with visit counters

LOS, SPECULAR, DIFFUSE, RECORD, TIMING, AVERAGE, DPS_LAUNCH, POLARIZED = 1, 2, 4, 8, 16, 32, 64, 128
STAGES = ("init", "trace", "keys", "refine", "diffuse_order", "diffuse", "los_combine")
CNT = dict(interactions=0, rays=1, segments=2, keys=3, specular=4, diffuse=5, status=6, candidates=7,
           tie_spill=8, trace_nodes=9, trace_disks=10, refine_nodes=11, refine_disks=12, diffuse_nodes=13,
           diffuse_disks=14, diffuse_occluded_nodes=15)
KAPPA_NONE = 0xFFFFFFFF


class PcrtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("pcrt error %d: %s" % (code, msg))
        self.code = code


class Points(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("normal", ctypes.c_void_p), ("material", ctypes.c_void_p),
                ("surface", ctypes.c_void_p), ("n_points", ctypes.c_uint32), ("disk_radius", ctypes.c_float)]


class BvhOpts(ctypes.Structure):
    _fields_ = [("leaf_size", ctypes.c_uint32), ("width", ctypes.c_uint32), ("builder", ctypes.c_uint32),
                ("dps_voxel", ctypes.c_float)]


BUILD_LBVH, BUILD_PLOC = 1, 2


class SceneInfo(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_uint32), ("n_surfaces", ctypes.c_uint32), ("n_materials", ctypes.c_uint32),
                ("depth", ctypes.c_uint32), ("n_nodes", ctypes.c_uint32), ("leaf_size", ctypes.c_uint32),
                ("width", ctypes.c_uint32), ("stack_entries", ctypes.c_uint32), ("builder", ctypes.c_uint32),
                ("bbox", ctypes.c_float * 6), ("build_ms", ctypes.c_double), ("n_point_sets", ctypes.c_uint32),
                ("dps_voxel", ctypes.c_float)]


class Thresholds(ctypes.Structure):
    _fields_ = [("eps_tie", ctypes.c_float), ("eps_self", ctypes.c_float), ("t_a_deg", ctypes.c_float),
                ("t_d", ctypes.c_float), ("kappa", ctypes.c_uint32)]


class SolveParams(ctypes.Structure):
    _fields_ = [("tx", ctypes.c_float * 3), ("rx", ctypes.c_void_p), ("n_rx", ctypes.c_uint32),
                ("freq_hz", ctypes.c_double), ("n_rays", ctypes.c_uint32), ("max_interactions", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("ray_subset", ctypes.c_void_p), ("n_subset", ctypes.c_uint32),
                ("thr", Thresholds), ("key_capacity", ctypes.c_uint32), ("wave_rays", ctypes.c_uint32),
                ("lambda_d", ctypes.c_float), ("dps_vis", ctypes.c_void_p), ("pol_tx", ctypes.c_float * 3),
                ("pol_rx", ctypes.c_float * 3)]


class Edge(ctypes.Structure):
    _fields_ = [("a", ctypes.c_float * 3), ("b", ctypes.c_float * 3), ("n0", ctypes.c_float * 3),
                ("n1", ctypes.c_float * 3), ("label0", ctypes.c_uint16), ("label1", ctypes.c_uint16)]


class BatchItem(ctypes.Structure):
    _fields_ = [("tx", ctypes.c_float * 3), ("n_rays", ctypes.c_uint32)]


class Tuning(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_uint32), ("leaf_size", ctypes.c_uint32), ("width", ctypes.c_uint32),
                ("wave_rays", ctypes.c_uint32), ("ms", ctypes.c_double)]


class Mlp(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p), ("b", ctypes.c_void_p), ("emb", ctypes.c_void_p), ("n_labels", ctypes.c_uint32)]


class Tape(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_uint32), ("n_trace_slots", ctypes.c_uint32), ("key_capacity", ctypes.c_uint32),
                ("label", ctypes.c_void_p), ("cos", ctypes.c_void_p), ("coef", ctypes.c_void_p),
                ("adj", ctypes.c_void_p)]


class Outputs(ctypes.Structure):
    _fields_ = [("gain", ctypes.c_void_p), ("h_te", ctypes.c_void_p), ("h_tm", ctypes.c_void_p),
                ("gain_parts", ctypes.c_void_p), ("ray_seq", ctypes.c_void_p), ("counters", ctypes.c_void_p)]


_lib = None
_libs = {}
_active = [None]


def use_counting(on: bool):
    """Route subsequent calls through the instrumented build (visit counters)."""
    _active[0] = "count" if on else None


def lib(variant=None) -> ctypes.CDLL:
    """The loaded libpcrt.so; raises if it has not been built."""
    global _lib
    variant = variant or _active[0] or "prod"
    if variant not in _libs:
        path = LIB_COUNT_PATH if variant == "count" else LIB_PATH
        if not os.path.exists(path):
            raise ImportError("%s is not built (run paper_2507_04021_amd/build.py or "
                              "__graft_entry__.build()); there is no fallback path" % os.path.basename(path))
        L = ctypes.CDLL(path)
        vp, u32, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_size_t
        L.pcrt_last_error.restype = ctypes.c_char_p
        L.pcrt_version.restype = ctypes.c_char_p
        L.pcrt_scene_workspace_size.argtypes = [u32, ctypes.POINTER(BvhOpts), ctypes.POINTER(sz)]
        L.pcrt_scene_create.argtypes = [ctypes.POINTER(Points), ctypes.POINTER(BvhOpts), vp, sz, vp,
                                        ctypes.POINTER(vp)]
        L.pcrt_scene_get_info.argtypes = [vp, ctypes.POINTER(SceneInfo)]
        L.pcrt_scene_destroy.argtypes = [vp]
        L.pcrt_reception_points.argtypes = [vp, vp, vp]
        L.pcrt_diffraction_workspace_size.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(sz)]
        L.pcrt_diffraction.argtypes = [vp, vp, ctypes.c_uint32, vp, ctypes.c_uint32, ctypes.POINTER(ctypes.c_float),
                                       vp, ctypes.c_uint32, ctypes.c_double, ctypes.c_float, vp, sz, vp, vp, vp]
        L.pcrt_diffraction_noalloc.argtypes = [vp, vp, ctypes.c_uint32, vp, ctypes.c_uint32,
                                               ctypes.POINTER(ctypes.c_float), vp, ctypes.c_uint32, ctypes.c_double,
                                               ctypes.c_float, vp, vp, vp]
        L.pcrt_visibility_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
        L.pcrt_visibility.argtypes = [vp, vp, ctypes.c_uint32, ctypes.c_float, vp, sz, vp, vp]
        L.pcrt_solve_workspace_size.argtypes = [vp, ctypes.POINTER(SolveParams), ctypes.POINTER(sz)]
        L.pcrt_solve.argtypes = [vp, vp, u32, ctypes.POINTER(SolveParams), vp, sz, ctypes.POINTER(Outputs), vp]
        L.pcrt_paths_copy.argtypes = [vp, ctypes.POINTER(SolveParams), vp, u32, vp, vp, vp, vp, vp, vp, vp,
                                      ctypes.POINTER(u32), vp]
        L.pcrt_diffuse_vis_copy.argtypes = [vp, ctypes.POINTER(SolveParams), vp, vp, vp]
        L.pcrt_raygen.argtypes = [u32, vp, u32, vp, vp]
        L.pcrt_stage_times.argtypes = [ctypes.POINTER(ctypes.c_double), u32]
        L.pcrt_status_poll.argtypes = [vp]
        L.pcrt_batch_workspace_size.argtypes = [vp, ctypes.POINTER(SolveParams), vp, u32, ctypes.POINTER(sz)]
        L.pcrt_solve_batch.argtypes = [vp, vp, u32, ctypes.POINTER(SolveParams), vp, u32, vp, sz,
                                       ctypes.POINTER(Outputs), vp]
        L.pcrt_graph_capture_batch.argtypes = [vp, vp, u32, ctypes.POINTER(SolveParams), vp, u32, vp, sz,
                                               ctypes.POINTER(Outputs), vp, ctypes.POINTER(vp)]
        L.pcrt_graph_launch.argtypes = [vp, vp]
        L.pcrt_graph_destroy.argtypes = [vp]
        L.pcrt_autotune.argtypes = [ctypes.POINTER(vp), u32, ctypes.POINTER(SolveParams), vp, u32, vp, u32, u32, vp,
                                    sz, ctypes.POINTER(Outputs), vp, vp, ctypes.POINTER(Tuning)]
        L.pcrt_mlp_forward.argtypes = [ctypes.POINTER(Mlp), u32, vp, vp, ctypes.c_float, vp, vp]
        L.pcrt_mlp_workspace_size.argtypes = [u32, u32, ctypes.POINTER(sz)]
        L.pcrt_mlp_backward.argtypes = [ctypes.POINTER(Mlp), u32, vp, vp, ctypes.c_float, vp, vp, sz, vp, vp, vp, vp]
        L.pcrt_tape_get.argtypes = [vp, ctypes.POINTER(SolveParams), vp, ctypes.POINTER(Tape)]
        L.pcrt_tape_fresnel.argtypes = [vp, ctypes.POINTER(SolveParams), vp, vp, u32, vp]
        L.pcrt_tape_forward.argtypes = [vp, ctypes.POINTER(SolveParams), vp, ctypes.POINTER(Outputs), vp]
        L.pcrt_tape_backward.argtypes = [vp, ctypes.POINTER(SolveParams), vp, vp, vp]
        L.pcrt_material_grad.argtypes = [vp, ctypes.POINTER(SolveParams), vp, vp, u32, vp, vp]
        L.pcrt_tape_cfr.argtypes = [vp, ctypes.POINTER(SolveParams), vp, ctypes.c_double, u32, vp, vp]
        L.pcrt_tape_cfr_backward.argtypes = [vp, ctypes.POINTER(SolveParams), vp, ctypes.c_double, u32, vp, vp]
        _libs[variant] = L
        if variant == "prod":
            _lib = L
    return _libs[variant]


def _check(rc, L=None):
    if rc != 0:
        raise PcrtError(rc, (L or lib()).pcrt_last_error().decode())


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(a, dtype, device):
    torch = _torch()
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Scene:
    """A point cloud of disks with its bounding-volume hierarchy on the GPU."""

    def __init__(self, pos, normal, material, surface, radius, leaf_size=4, width=4, builder=0, device="cuda",
                 stream=None, dps_voxel=0.0):
        """dps_voxel > 0 also groups the points into voxels of that edge (the point
        sets of the AVERAGE solves)."""
        torch = _torch()
        self.device = torch.device(device)
        pos = _dev(pos, torch.float32, self.device).reshape(-1, 3)
        nrm = _dev(normal, torch.float32, self.device).reshape(-1, 3)
        mat = _dev(np.asarray(material, np.int32) if not isinstance(material, torch.Tensor) else material,
                   torch.int32, self.device).to(torch.int16)
        surf = _dev(np.asarray(surface, np.int64) if not isinstance(surface, torch.Tensor) else surface,
                    torch.int64, self.device).to(torch.int32)
        n = pos.shape[0]
        self.n = n
        self.radius = float(radius)
        opts = BvhOpts(leaf_size, width, builder, float(dps_voxel))
        nbytes = ctypes.c_size_t(0)
        _check(lib().pcrt_scene_workspace_size(n, ctypes.byref(opts), ctypes.byref(nbytes)))
        self.ws = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=self.device)
        pts = Points(pos.data_ptr(), nrm.data_ptr(), mat.data_ptr(), surf.data_ptr(), n, radius)
        h = ctypes.c_void_p()
        self._variant = _active[0] or "prod"
        _check(lib().pcrt_scene_create(ctypes.byref(pts), ctypes.byref(opts), _ptr(self.ws), nbytes.value,
                                       _stream(stream), ctypes.byref(h)))
        self.handle = h
        info = SceneInfo()
        _check(lib().pcrt_scene_get_info(self.handle, ctypes.byref(info)))
        self.info = dict(n_points=info.n_points, n_surfaces=info.n_surfaces, n_materials=info.n_materials,
                         depth=info.depth, n_nodes=info.n_nodes, leaf_size=info.leaf_size, width=info.width,
                         stack_entries=info.stack_entries, builder=info.builder, bbox=list(info.bbox),
                         build_ms=info.build_ms, n_point_sets=info.n_point_sets, dps_voxel=info.dps_voxel)

    @classmethod
    def from_scene(cls, sc, **kw):
        """From a scenes.Scene (numpy arrays)."""
        return cls(sc.pos, sc.normal, sc.material.astype(np.int32), sc.surface.astype(np.int64), sc.radius, **kw)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _libs:
            lib(self._variant).pcrt_scene_destroy(h)
            self.handle = None


def reception_points(scene: Scene, stream=None):
    """float32[n_point_sets, 3] device tensor: the mean centre of each point set."""
    torch = _torch()
    L = lib(scene._variant)
    out = torch.empty(max(scene.info["n_point_sets"], 1), 3, dtype=torch.float32, device=scene.device)
    _check(L.pcrt_reception_points(scene.handle, _ptr(out), _stream(stream)), L)
    return out[:scene.info["n_point_sets"]]


def visibility(scene: Scene, rx, eps_self=0.0, ws=None, out=None, stream=None):
    """uint8[n_rx, n_point_sets] device tensor: 1 where the receiver sees the
    set's reception point (the set's own disks aside)."""
    torch = _torch()
    L = lib(scene._variant)
    rx_t = _dev(np.asarray(rx, np.float32).reshape(-1, 3) if not isinstance(rx, torch.Tensor) else rx,
                torch.float32, scene.device).reshape(-1, 3)
    nb = ctypes.c_size_t(0)
    _check(L.pcrt_visibility_workspace_size(scene.handle, ctypes.byref(nb)), L)
    if ws is None or ws.numel() < nb.value:
        ws = torch.empty(nb.value, dtype=torch.uint8, device=scene.device)
    n = scene.info["n_point_sets"]
    if out is None:
        out = torch.empty(rx_t.shape[0], max(n, 1), dtype=torch.uint8, device=scene.device)
    _check(L.pcrt_visibility(scene.handle, _ptr(rx_t), rx_t.shape[0], float(eps_self), _ptr(ws), ws.numel(),
                             _ptr(out), _stream(stream)), L)
    return out[:, :n]


def edges_tensor(rows, labels, device="cuda"):
    """Device array of pcrt_edge from rows float[n, 12] (a, b, n0, n1) and labels int[n, 2]."""
    torch = _torch()
    rows = np.ascontiguousarray(rows, np.float32).reshape(-1, 12)
    labels = np.ascontiguousarray(labels, np.int64).reshape(-1, 2)
    arr = (Edge * len(rows))()
    for i in range(len(rows)):
        arr[i].a[:] = rows[i, 0:3].tolist()
        arr[i].b[:] = rows[i, 3:6].tolist()
        arr[i].n0[:] = rows[i, 6:9].tolist()
        arr[i].n1[:] = rows[i, 9:12].tolist()
        arr[i].label0, arr[i].label1 = int(labels[i, 0]), int(labels[i, 1])
    raw = np.frombuffer(bytes(arr), np.uint8)
    return torch.as_tensor(raw.copy(), device=device), len(rows)


def diffraction(scene: Scene, edges, mats, tx, rx, freq, eps_self=0.0, want_pairs=False, ws=None, stream=None):
    """Single-bounce diffracted paths over edges (from edges_tensor, or (rows, labels)).
    Returns (out float64[n_rx, 5]: G, h_TE re, im, h_TM re, im; pair amplitudes complex
    [n_rx, n_edges, 2] or None)."""
    torch = _torch()
    L = lib(scene._variant)
    dev = scene.device
    e_t, n_e = edges if isinstance(edges, tuple) and isinstance(edges[0], torch.Tensor) else \
        edges_tensor(edges[0], edges[1], dev)
    mats_t = mats if isinstance(mats, torch.Tensor) and mats.device.type == "cuda" else materials_tensor(mats, dev)
    rx_t = _dev(np.asarray(rx, np.float32).reshape(-1, 3) if not isinstance(rx, torch.Tensor) else rx,
                torch.float32, dev).reshape(-1, 3)
    n_rx = rx_t.shape[0]
    nb = ctypes.c_size_t(0)
    _check(L.pcrt_diffraction_workspace_size(scene.handle, n_e, n_rx, ctypes.byref(nb)), L)
    if ws is None or ws.numel() < nb.value:
        ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    out = torch.empty(n_rx, 5, dtype=torch.float64, device=dev)
    pairs = torch.empty(n_rx, n_e, 4, dtype=torch.float32, device=dev) if want_pairs else None
    txa = (ctypes.c_float * 3)(*[float(v) for v in np.asarray(tx, np.float32).reshape(3)])
    _check(L.pcrt_diffraction(scene.handle, _ptr(e_t), n_e, _ptr(mats_t), mats_t.shape[0], txa, _ptr(rx_t), n_rx,
                              float(freq), float(eps_self), _ptr(ws), ws.numel(), _ptr(out), _ptr(pairs),
                              _stream(stream)), L)
    amp = None
    if want_pairs:
        p = pairs.cpu().numpy().astype(np.float64)
        amp = np.stack([p[..., 0] + 1j * p[..., 1], p[..., 2] + 1j * p[..., 3]], -1)
    return out, amp


def materials_tensor(mats, device="cuda"):
    """float32[n_labels, 3] (eps_r, sigma, S) on the device."""
    torch = _torch()
    if isinstance(mats, torch.Tensor):
        return mats.detach().to(device=device, dtype=torch.float32).reshape(-1, 3).contiguous()
    return _dev(np.asarray(mats, np.float64).reshape(-1, 3), torch.float32, device)


@dataclass
class SolveResult:
    gain: object           # float64[n_rx]
    h_te: object           # complex as float64[n_rx, 2]
    h_tm: object
    parts: object          # float64[n_rx, 3] (los, specular, diffuse)
    seq: object            # int32[n_trace, K] or None
    counters: object       # uint64[16] as int64
    ws: object             # the workspace (holds the tape of a RECORD solve)
    params: SolveParams
    scene: Scene
    keep: tuple            # device tensors the params point to

    def counter(self, name):
        return int(self.counters[CNT[name]].item())

    def fetch_status(self, stream=None):
        """Start copying the counters to pinned host memory without waiting;
        check_status() then waits only for this copy."""
        torch = _torch()
        self._status_host = torch.empty(16, dtype=torch.int64, pin_memory=True)
        self._status_host.copy_(self.counters, non_blocking=True)
        self._status_event = torch.cuda.Event()
        self._status_event.record(stream if stream is not None else torch.cuda.current_stream())

    def check_status(self):
        """Raise PcrtError if the solve's device status word has a bit set
        (key table overflow, invalid material label, tape capacity exceeded).
        Waits for the solve (or for the copy fetch_status started)."""
        if getattr(self, "_status_ok", False):
            return
        if getattr(self, "_status_event", None) is not None:
            self._status_event.synchronize()
            host = self._status_host.numpy().astype(np.uint64)
        else:
            host = np.ascontiguousarray(self.counters.cpu().numpy().astype(np.uint64))
        L = lib(self.scene._variant)
        _check(L.pcrt_status_poll(np.ascontiguousarray(host).ctypes.data_as(ctypes.c_void_p)), L)
        self._status_ok = True


def make_params(tx, rx_t, freq, n_rays, K, flags, subset_t=None, thr=None, key_capacity=0, wave_rays=0,
                lambda_d=0.0, dps_vis=None):
    th = Thresholds(0.0, 0.0, 0.0, 0.0, 0)
    if thr:
        for k, v in thr.items():
            setattr(th, k, v)
    p = SolveParams()
    p.tx = (ctypes.c_float * 3)(*[float(v) for v in np.asarray(tx, np.float32).reshape(3)])
    p.rx = rx_t.data_ptr()
    p.n_rx = rx_t.shape[0]
    p.freq_hz = float(freq)
    p.n_rays = int(n_rays)
    p.max_interactions = int(K)
    p.flags = int(flags)
    p.ray_subset = subset_t.data_ptr() if subset_t is not None else None
    p.n_subset = subset_t.numel() if subset_t is not None else 0
    p.thr = th
    p.key_capacity = int(key_capacity)
    p.wave_rays = int(wave_rays)
    p.lambda_d = float(lambda_d)
    p.dps_vis = dps_vis.data_ptr() if dps_vis is not None else None
    return p


def solve(scene: Scene, mats, tx, rx, freq, n_rays, K=2, flags=LOS | SPECULAR, ray_subset=None, thr=None,
          want_seq=False, stream=None, ws=None, out=None, key_capacity=0, wave_rays=0,
          lambda_d=0.0, dps_vis=None, pol=None) -> SolveResult:
    """One transmitter against all receivers. mats: (n_labels, 3) or a device tensor from materials_tensor.
    flags with AVERAGE: point-set averaged interactions (scene built with dps_voxel > 0), depth
    attenuation lambda_d (0 = 100 per metre). flags with DPS_LAUNCH: one ray per point set towards its
    reception point (n_rays = the scene's n_point_sets) and specular candidates gated by dps_vis
    (the uint8[n_rx, n_point_sets] tensor from visibility() for the same receivers).
    pol = (pol_tx, pol_rx): the polarised (Jones-vector) field of line-of-sight and specular paths for
    these transmit and receive polarisation vectors (sets POLARIZED)."""
    torch = _torch()
    L = lib(scene._variant)
    dev = scene.device
    mats_t = mats if isinstance(mats, torch.Tensor) and mats.device.type == "cuda" else materials_tensor(mats, dev)
    rx_t = _dev(np.asarray(rx, np.float32).reshape(-1, 3) if not isinstance(rx, torch.Tensor) else rx,
                torch.float32, dev).reshape(-1, 3)
    sub_t = None
    if ray_subset is not None:
        sub_t = _dev(np.asarray(ray_subset, np.int64).astype(np.int32) if not isinstance(ray_subset, torch.Tensor)
                     else ray_subset, torch.int32, dev)
    if dps_vis is not None:
        dps_vis = dps_vis.contiguous()
    if pol is not None:
        flags |= POLARIZED
    p = make_params(tx, rx_t, freq, n_rays, K, flags, sub_t, thr, key_capacity, wave_rays, lambda_d, dps_vis)
    if pol is not None:
        p.pol_tx[:] = [float(v) for v in np.asarray(pol[0], np.float32).reshape(3)]
        p.pol_rx[:] = [float(v) for v in np.asarray(pol[1], np.float32).reshape(3)]
    nbytes = ctypes.c_size_t(0)
    _check(L.pcrt_solve_workspace_size(scene.handle, ctypes.byref(p), ctypes.byref(nbytes)), L)
    if ws is None or ws.numel() < nbytes.value:
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
    n_rx = rx_t.shape[0]
    if out is None:
        n_trace = 0 if not (flags & (SPECULAR | DIFFUSE)) else (sub_t.numel() if sub_t is not None else n_rays)
        out = dict(gain=torch.empty(n_rx, dtype=torch.float64, device=dev),
                   h_te=torch.empty(n_rx, 2, dtype=torch.float64, device=dev),
                   h_tm=torch.empty(n_rx, 2, dtype=torch.float64, device=dev),
                   parts=torch.empty(n_rx, 3, dtype=torch.float64, device=dev),
                   seq=torch.empty(max(n_trace, 1), K, dtype=torch.int32, device=dev) if want_seq else None,
                   counters=torch.empty(16, dtype=torch.int64, device=dev))
    o = Outputs(out["gain"].data_ptr(), out["h_te"].data_ptr(), out["h_tm"].data_ptr(), out["parts"].data_ptr(),
                out["seq"].data_ptr() if out.get("seq") is not None else None, out["counters"].data_ptr())
    _check(L.pcrt_solve(scene.handle, _ptr(mats_t), mats_t.shape[0], ctypes.byref(p), _ptr(ws), ws.numel(),
                        ctypes.byref(o), _stream(stream)), L)
    return SolveResult(out["gain"], out["h_te"], out["h_tm"], out["parts"], out.get("seq"), out["counters"], ws, p,
                       scene, (mats_t, rx_t, sub_t, dps_vis))


def paths(res: SolveResult, stream=None):
    """Specular path list of a RECORD solve as numpy arrays."""
    torch = _torch()
    L = lib(res.scene._variant)
    res.check_status()
    p = res.params
    K, n_rx = p.max_interactions, p.n_rx
    nk = ctypes.c_uint32(0)
    _check(L.pcrt_paths_copy(res.scene.handle, ctypes.byref(p), _ptr(res.ws), 0, None, None, None, None, None,
                                 None, None, ctypes.byref(nk), _stream(stream)), L)
    n = max(nk.value, 1)
    dev = res.scene.device
    key_ray = torch.empty(n, dtype=torch.int32, device=dev)
    key_len = torch.empty(n, dtype=torch.uint8, device=dev)
    key_seq = torch.empty(n, K, dtype=torch.int32, device=dev)
    valid = torch.empty(n, n_rx, dtype=torch.uint8, device=dev)
    length = torch.empty(n, n_rx, dtype=torch.float32, device=dev)
    amp = torch.empty(n, n_rx, 4, dtype=torch.float32, device=dev)
    hit = torch.empty(n, n_rx, K, dtype=torch.int32, device=dev)
    _check(L.pcrt_paths_copy(res.scene.handle, ctypes.byref(p), _ptr(res.ws), nk.value, _ptr(key_ray),
                                 _ptr(key_len), _ptr(key_seq), _ptr(valid), _ptr(length), _ptr(amp), _ptr(hit),
                                 ctypes.byref(nk), _stream(stream)), L)
    m = nk.value
    a = amp[:m].cpu().numpy()
    return dict(n_keys=m, key_ray=key_ray[:m].cpu().numpy(), key_len=key_len[:m].cpu().numpy(),
                key_seq=key_seq[:m].cpu().numpy(), valid=valid[:m].cpu().numpy().astype(bool),
                length=length[:m].cpu().numpy(), amp_te=a[..., 0] + 1j * a[..., 1], amp_tm=a[..., 2] + 1j * a[..., 3],
                hit=hit[:m].cpu().numpy())


def diffuse_vis(res: SolveResult, stream=None):
    torch = _torch()
    L = lib(res.scene._variant)
    p = res.params
    n_trace = p.n_subset if p.ray_subset else p.n_rays
    vis = torch.empty(n_trace, p.max_interactions, p.n_rx, dtype=torch.uint8, device=res.scene.device)
    _check(L.pcrt_diffuse_vis_copy(res.scene.handle, ctypes.byref(p), _ptr(res.ws), _ptr(vis), _stream(stream)), L)
    return vis


# ------------------------------------------------------------------ batch
@dataclass
class BatchResult:
    gain: object      # float64[n_items, n_rx]
    h_te: object      # float64[n_items, n_rx, 2]
    h_tm: object
    parts: object     # float64[n_items, n_rx, 3]
    counters: object
    ws: object
    params: SolveParams
    items: object     # ctypes array of BatchItem
    keep: tuple

    def counter(self, name):
        return int(self.counters[CNT[name]].item())


def _items(tx, n_rays):
    tx = np.asarray(tx, np.float32).reshape(-1, 3)
    n_rays = np.broadcast_to(np.asarray(n_rays, np.int64), (tx.shape[0],))
    arr = (BatchItem * tx.shape[0])()
    for i in range(tx.shape[0]):
        arr[i].tx = (ctypes.c_float * 3)(*[float(v) for v in tx[i]])
        arr[i].n_rays = int(n_rays[i])
    return arr


def _batch_setup(scene, mats, tx, n_rays, rx, freq, K, flags, thr, wave_rays, lambda_d=0.0):
    torch = _torch()
    dev = scene.device
    mats_t = mats if isinstance(mats, torch.Tensor) and mats.device.type == "cuda" else materials_tensor(mats, dev)
    rx_t = _dev(np.asarray(rx, np.float32).reshape(-1, 3) if not isinstance(rx, torch.Tensor) else rx,
                torch.float32, dev).reshape(-1, 3)
    items = _items(tx, n_rays)
    p = make_params([0, 0, 0], rx_t, freq, 1, K, flags, None, thr, 0, wave_rays, lambda_d)
    L = lib(scene._variant)
    nbytes = ctypes.c_size_t(0)
    _check(L.pcrt_batch_workspace_size(scene.handle, ctypes.byref(p), items, len(items), ctypes.byref(nbytes)), L)
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
    n, r = len(items), rx_t.shape[0]
    out = dict(gain=torch.empty(n, r, dtype=torch.float64, device=dev),
               h_te=torch.empty(n, r, 2, dtype=torch.float64, device=dev),
               h_tm=torch.empty(n, r, 2, dtype=torch.float64, device=dev),
               parts=torch.empty(n, r, 3, dtype=torch.float64, device=dev),
               counters=torch.empty(16, dtype=torch.int64, device=dev))
    o = Outputs(out["gain"].data_ptr(), out["h_te"].data_ptr(), out["h_tm"].data_ptr(), out["parts"].data_ptr(),
                None, out["counters"].data_ptr())
    return L, mats_t, rx_t, items, p, ws, out, o


def solve_batch(scene: Scene, mats, tx, n_rays, rx, freq, K=2, flags=LOS | SPECULAR, thr=None, wave_rays=0,
                stream=None, lambda_d=0.0) -> BatchResult:
    """Many transmitters (tx[n, 3], n_rays[n]) against the same receivers in one launch sequence."""
    L, mats_t, rx_t, items, p, ws, out, o = _batch_setup(scene, mats, tx, n_rays, rx, freq, K, flags, thr,
                                                         wave_rays, lambda_d)
    _check(L.pcrt_solve_batch(scene.handle, _ptr(mats_t), mats_t.shape[0], ctypes.byref(p), items, len(items),
                              _ptr(ws), ws.numel(), ctypes.byref(o), _stream(stream)), L)
    return BatchResult(out["gain"], out["h_te"], out["h_tm"], out["parts"], out["counters"], ws, p, items,
                       (mats_t, rx_t, o))


class BatchGraph:
    """A batch solve captured once as a HIP graph (by the library) and
    replayed. Materials may be changed in place in `self.mats` between
    launches; outputs land in the same tensors every launch."""

    def __init__(self, scene: Scene, mats, tx, n_rays, rx, freq, K=2, flags=LOS | SPECULAR, thr=None, wave_rays=0,
                 stream=None):
        torch = _torch()
        self.scene = scene
        self.stream = stream if stream is not None else torch.cuda.Stream()
        (self.L, self.mats, self.rx, self.items, self.params, self.ws, self.out,
         self._o) = _batch_setup(scene, mats, tx, n_rays, rx, freq, K, flags, thr, wave_rays)
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        _check(self.L.pcrt_graph_capture_batch(scene.handle, _ptr(self.mats), self.mats.shape[0],
                                               ctypes.byref(self.params), self.items, len(self.items), _ptr(self.ws),
                                               self.ws.numel(), ctypes.byref(self._o), _stream(self.stream),
                                               ctypes.byref(h)), self.L)
        self.handle = h

    def launch(self, stream=None):
        s = stream if stream is not None else self.stream
        _check(self.L.pcrt_graph_launch(self.handle, _stream(s)), self.L)
        return self.out

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None:
            self.L.pcrt_graph_destroy(h)
            self.handle = None


def autotune(sc, mats, tx, rx, freq, n_rays, K=2, flags=LOS | SPECULAR, leaf_sizes=(1, 2, 4, 8), widths=(2, 4, 8),
             wave_rays=(64, 128, 256), builders=(0,), reps=3, cache_path=None, device="cuda"):
    """Sweep BVH builder x leaf size x node width x rays per wavefront fetch
    with the library's tuner (one scene per builder, leaf size and width,
    built here); the winner is stored in a JSON cache keyed by the workload."""
    import hashlib
    import json
    torch = _torch()
    # the cached choice is only valid for the same library build and candidate sets
    with open(LIB_PATH, "rb") as f:
        build_id = hashlib.sha1(f.read()).hexdigest()[:16]
    key = "n=%d rays=%d K=%d flags=%d rx=%d dev=%s lib=%s cands=%s" % (
        sc.n, n_rays, K, flags, np.asarray(rx).reshape(-1, 3).shape[0], torch.cuda.get_device_name(device), build_id,
        repr((tuple(builders), tuple(leaf_sizes), tuple(widths), tuple(wave_rays), reps)))
    cache_path = cache_path or os.path.join(os.path.expanduser("~"), ".cache", "pcrt_tuning.json")
    try:
        cache = json.load(open(cache_path))
    except (OSError, ValueError):
        cache = {}
    if key in cache:
        return cache[key], None
    L = lib()
    cands = [Scene.from_scene(sc, leaf_size=l, width=w, builder=b, device=device)
             for b in builders for l in leaf_sizes for w in widths]
    res = solve(cands[0], mats, tx, rx, freq, n_rays, K=K, flags=flags)
    p = res.params
    need = 0
    for c in cands:
        for wr_ in wave_rays:
            q = SolveParams.from_buffer_copy(p)
            q.wave_rays = wr_
            nb = ctypes.c_size_t(0)
            _check(L.pcrt_solve_workspace_size(c.handle, ctypes.byref(q), ctypes.byref(nb)), L)
            need = max(need, nb.value)
    ws = torch.empty(need, dtype=torch.uint8, device=torch.device(device))
    o = Outputs(res.gain.data_ptr(), res.h_te.data_ptr(), res.h_tm.data_ptr(), res.parts.data_ptr(), None,
                res.counters.data_ptr())
    handles = (ctypes.c_void_p * len(cands))(*[c.handle.value for c in cands])
    wr = (ctypes.c_uint32 * len(wave_rays))(*wave_rays)
    table = (Tuning * (len(cands) * len(wave_rays)))()
    best = Tuning()
    mats_t = res.keep[0]
    _check(L.pcrt_autotune(handles, len(cands), ctypes.byref(p), _ptr(mats_t), mats_t.shape[0], wr, len(wave_rays),
                           reps, _ptr(ws), ws.numel(), ctypes.byref(o), _stream(), table, ctypes.byref(best)), L)
    choice = dict(builder=cands[best.scene].info["builder"], leaf_size=best.leaf_size, width=best.width,
                  wave_rays=best.wave_rays, ms=best.ms)
    rows = [dict(builder=cands[t.scene].info["builder"], leaf_size=t.leaf_size, width=t.width, wave_rays=t.wave_rays,
                 ms=t.ms) for t in table]
    cache[key] = choice
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        json.dump(cache, open(cache_path, "w"), indent=1)
    except OSError:
        pass
    return choice, rows


# ------------------------------------------------------------------ tape
def tape(res: SolveResult):
    """Device views of a RECORD solve's tape: dict of torch tensors (label,
    cos, coef [n_slots, 8], adj [n_slots, 8]) and sizes."""
    torch = _torch()
    L = lib(res.scene._variant)
    res.check_status()  # once per recording: a tape with dropped paths is refused
    t = Tape()
    _check(L.pcrt_tape_get(res.scene.handle, ctypes.byref(res.params), _ptr(res.ws), ctypes.byref(t)), L)
    base = res.ws.data_ptr()
    n = t.n_slots

    def view(ptr, nbytes, dtype, shape):
        off = ptr - base
        return res.ws[off:off + nbytes].view(dtype).reshape(shape)

    return dict(n_slots=n, n_trace_slots=t.n_trace_slots, key_capacity=t.key_capacity,
                label=view(t.label, 2 * n, torch.int16, (n,)), cos=view(t.cos, 4 * n, torch.float32, (n,)),
                coef=view(t.coef, 32 * n, torch.float32, (n, 8)), adj=view(t.adj, 32 * n, torch.float32, (n, 8)))


def tape_fresnel(res: SolveResult, mats, stream=None):
    """Fill the tape's coefficient rows from per-label materials (n_labels, 3)."""
    L = lib(res.scene._variant)
    m = materials_tensor(mats, res.scene.device)
    _check(L.pcrt_tape_fresnel(res.scene.handle, ctypes.byref(res.params), _ptr(res.ws), _ptr(m), m.shape[0],
                               _stream(stream)), L)
    return m


def tape_forward(res: SolveResult, stream=None):
    """Per-receiver gain (float64 tensor) from the tape's coefficient rows."""
    torch = _torch()
    L = lib(res.scene._variant)
    n = res.params.n_rx
    dev = res.scene.device
    g = torch.empty(n, dtype=torch.float64, device=dev)
    h_te = torch.empty(n, 2, dtype=torch.float64, device=dev)
    h_tm = torch.empty(n, 2, dtype=torch.float64, device=dev)
    parts = torch.empty(n, 3, dtype=torch.float64, device=dev)
    o = Outputs(g.data_ptr(), h_te.data_ptr(), h_tm.data_ptr(), parts.data_ptr(), None, None)
    _check(L.pcrt_tape_forward(res.scene.handle, ctypes.byref(res.params), _ptr(res.ws), ctypes.byref(o),
                               _stream(stream)), L)
    return g, h_te, h_tm, parts


def tape_backward(res: SolveResult, dl_dg, stream=None):
    """Adjoint rows of the tape for dL/dG (float64 [n_rx])."""
    torch = _torch()
    L = lib(res.scene._variant)
    d = dl_dg.to(device=res.scene.device, dtype=torch.float64).contiguous()
    _check(L.pcrt_tape_backward(res.scene.handle, ctypes.byref(res.params), _ptr(res.ws), _ptr(d),
                                _stream(stream)), L)
    return d


def tape_cfr(res: SolveResult, bandwidth_hz: float, n_freq: int, stream=None):
    """Channel frequency response of a RECORD solve's paths with the tape's
    current coefficient rows: complex128 [n_rx, n_freq, 2] (TE, TM) at n_freq
    equally spaced frequencies spanning bandwidth_hz around the solve's."""
    torch = _torch()
    L = lib(res.scene._variant)
    n_rx = res.params.n_rx
    out = torch.empty(n_rx, n_freq, 4, dtype=torch.float64, device=res.scene.device)
    _check(L.pcrt_tape_cfr(res.scene.handle, ctypes.byref(res.params), _ptr(res.ws), float(bandwidth_hz), int(n_freq),
                           _ptr(out), _stream(stream)), L)
    return torch.complex(out[..., 0::2], out[..., 1::2])


def tape_cfr_backward(res: SolveResult, bandwidth_hz: float, n_freq: int, dl_dh, stream=None):
    """Adjoint rows of the tape for dL/dH, given as a complex [n_rx, n_freq, 2]
    tensor dL/dRe + j dL/dIm of each sample."""
    torch = _torch()
    L = lib(res.scene._variant)
    g = dl_dh.to(device=res.scene.device, dtype=torch.complex128)
    d = torch.stack([g[..., 0].real, g[..., 0].imag, g[..., 1].real, g[..., 1].imag], -1).contiguous()
    _check(L.pcrt_tape_cfr_backward(res.scene.handle, ctypes.byref(res.params), _ptr(res.ws), float(bandwidth_hz),
                                    int(n_freq), _ptr(d), _stream(stream)), L)
    return d


def material_grad(res: SolveResult, mats_dev, stream=None):
    """dL/d(eps_r, sigma, S) per label (float64 [n_labels, 3]) from the adjoint rows."""
    torch = _torch()
    L = lib(res.scene._variant)
    out = torch.empty(mats_dev.shape[0], 3, dtype=torch.float64, device=res.scene.device)
    _check(L.pcrt_material_grad(res.scene.handle, ctypes.byref(res.params), _ptr(res.ws), _ptr(mats_dev),
                                mats_dev.shape[0], _ptr(out), _stream(stream)), L)
    return out


def stage_times():
    """Per-stage device ms of the last TIMING solve on this thread (synchronises)."""
    arr = (ctypes.c_double * len(STAGES))()
    _check(lib().pcrt_stage_times(arr, len(STAGES)))
    return dict(zip(STAGES, list(arr)))


def raygen(n_budget, ids=None, device="cuda", stream=None):
    torch = _torch()
    ids_t = None if ids is None else _dev(np.asarray(ids, np.int64).astype(np.int32), torch.int32, device)
    n = n_budget if ids is None else ids_t.numel()
    out = torch.empty(n, 3, dtype=torch.float32, device=device)
    _check(lib().pcrt_raygen(n_budget, _ptr(ids_t), n, _ptr(out), _stream(stream)))
    return out
