"""Python binding of the emrt C ABI: argument marshalling onto torch device
tensors.  Every step of the method runs in the HIP library; this module only
allocates device buffers (torch), passes pointers and reads results back."""
from __future__ import annotations

import ctypes
import json
import math
import os
from typing import Dict, Optional, Sequence

import numpy as np
import torch

from . import _abi as A


class EmrtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"emrt status {status}: {msg}")
        self.status = status


def _ptr(t: Optional[torch.Tensor]) -> int:
    return 0 if t is None else int(t.data_ptr())


def _numel(a) -> int:
    return a.numel() if isinstance(a, torch.Tensor) else np.asarray(a).size


def _dev(a, dtype, device) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device).contiguous()


class Tracer:
    """One emrt context bound to one scene, n_tx transmitters and n_rx receivers.

    ``scene`` provides ``verts, tris, tri_face, face_object, face_material,
    object_dynamic, materials`` (numpy or torch); ``config`` keys mirror
    ``emrt_config`` (freq_hz list, max_reflections, diffraction, rays_per_tx,
    rx_sphere_k, diff_max_leg_m, tx_power_w, antenna_mode, path_cap_per_link,
    path_capacity, table_capacity, adjoint_materials, dyn_rebuild_ratio, ray_regroup).
    """

    def __init__(self, scene, n_tx: int, n_rx: int, device: str = "cuda", static_workspace: bool = False, **config):
        self.lib = A.load()
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise RuntimeError("the emrt library runs on the GPU only")
        cfg = A.Config()
        self.lib.emrt_config_default(ctypes.byref(cfg))
        freqs = list(config.pop("freq_hz", [28e9]))
        cfg.n_freq = len(freqs)
        for i, f in enumerate(freqs[:4]):
            cfg.freq_hz[i] = float(f)
        for k, v in config.items():
            if not hasattr(cfg, k):
                raise TypeError(f"unknown config key {k}")
            setattr(cfg, k, v)
        self.cfg = cfg
        self.freqs = freqs
        self.n_tx, self.n_rx = int(n_tx), int(n_rx)
        self.n_links = self.n_tx * self.n_rx
        ctx = ctypes.c_void_p()
        self._check(self.lib.emrt_ctx_create(ctypes.byref(cfg), ctypes.byref(ctx)), None)
        self.ctx = ctx
        sz = A.Sizes(len(scene.verts), len(scene.tris), len(scene.face_object), len(scene.object_dynamic),
                     self.n_tx, self.n_rx)
        nbytes = ctypes.c_size_t()
        self._check(self.lib.emrt_workspace_size(self.ctx, ctypes.byref(sz), ctypes.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        self.stream = torch.cuda.current_stream(self.device)
        self._check(self.lib.emrt_set_stream(self.ctx, ctypes.c_void_p(self.stream.cuda_stream)))
        self._lib_stream = self.stream  # the stream the context works on (a Batch's while it is a member)
        if static_workspace:  # the library's own array (emrt_bind_static_workspace): nothing is allocated
            self.workspace = None
            self._check(self.lib.emrt_bind_static_workspace(self.ctx))
        else:
            self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
            self._check(self.lib.emrt_bind_workspace(self.ctx, ctypes.c_void_p(_ptr(self.workspace)), nbytes.value))
        # state generation: advanced by every call that changes what the
        # adjoint of the last step would differentiate (a step, a frame, the
        # materials), so a recorded forward can tell whether it is still current
        self.generation = 0
        self.set_scene(scene)
        self._frame_refs = None

    # ------------------------------------------------------------------ util
    def _check(self, st: int, ctx=0) -> int:
        if st < 0:
            msg = A.load().emrt_status_string(st).decode()
            if ctx is not None:
                buf = ctypes.create_string_buffer(512)
                self.lib.emrt_last_error(self.ctx, buf, 512)
                msg = buf.value.decode() or msg
            raise EmrtError(st, msg)
        return st

    def close(self) -> None:
        if getattr(self, "ctx", None):
            torch.cuda.synchronize(self.device)
            self.lib.emrt_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------------- scene
    def set_scene(self, sc) -> None:
        d = self.device
        self._scene_refs = dict(
            verts=_dev(sc.verts, torch.float32, d), tris=_dev(sc.tris, torch.int32, d),
            tri_face=_dev(sc.tri_face, torch.int32, d), face_object=_dev(sc.face_object, torch.int32, d),
            face_material=_dev(sc.face_material, torch.int32, d), object_dynamic=_dev(sc.object_dynamic, torch.uint8, d),
        )
        mats = np.asarray(sc.materials, np.complex128)
        self._mat_host = np.ascontiguousarray(np.stack([mats.real, mats.imag], 1), np.float64)
        r = self._scene_refs
        desc = A.SceneDesc(len(sc.verts), len(sc.tris), len(sc.face_object), len(sc.object_dynamic),
                           _ptr(r["verts"]), _ptr(r["tris"]), _ptr(r["tri_face"]), _ptr(r["face_object"]),
                           _ptr(r["face_material"]), _ptr(r["object_dynamic"]), len(mats),
                           self._mat_host.ctypes.data)
        self.n_dynamic = int(np.asarray(sc.object_dynamic).sum())
        self._check(self.lib.emrt_set_scene(self.ctx, ctypes.byref(desc)))
        refl = getattr(sc, "material_refl", None)
        if refl is not None:
            self.set_reflection_coefficients(refl)

    def set_reflection_coefficients(self, refl: Sequence[float]) -> None:
        """Per material: 0 = Fresnel from the permittivity, g in (0, 1] = a
        constant reflection coefficient of magnitude g (Table I)."""
        self.generation += 1
        self._refl_host = np.ascontiguousarray(np.asarray(refl, np.float64).reshape(-1))
        self._check(self.lib.emrt_set_reflection_coefficients(self.ctx, self._refl_host.ctypes.data,
                                                              len(self._refl_host)))

    def set_materials(self, eps: Sequence[complex]) -> None:
        self.generation += 1
        e = np.asarray(eps, np.complex128)
        self._mat_host = np.ascontiguousarray(np.stack([e.real, e.imag], 1), np.float64)
        self._check(self.lib.emrt_set_materials(self.ctx, self._mat_host.ctypes.data, len(e)))

    def set_frame(self, fr, frame_index: int = 0) -> None:
        self.generation += 1
        d = self.device
        nd = max(self.n_dynamic, 1)
        xf = np.zeros((nd, 3, 4)) if _numel(fr.obj_xform) == 0 else fr.obj_xform
        ov = np.zeros((nd, 3)) if _numel(fr.obj_vel) == 0 else fr.obj_vel
        arrays = dict(xf=xf, ov=ov, tx=fr.tx_pos, txv=fr.tx_vel, txo=fr.tx_orient, rx=fr.rx_pos, rxv=fr.rx_vel)
        if any(isinstance(v, torch.Tensor) for v in arrays.values()):
            refs = {k: _dev(v, torch.float64, d) for k, v in arrays.items()}
            ptrs = {k: _ptr(v) for k, v in refs.items()}
            self._frame_refs = refs  # kept alive until the next frame (stream order)
            entry = self.lib.emrt_set_frame
        else:
            # host arrays: the library packs them into its pinned buffer and
            # uploads them in one copy (emrt_set_frame_host).  Waiting first for
            # the work already queued keeps the host at most one step ahead of
            # the GPU, as a copy from pageable memory would: with several
            # discovery steps queued behind each other the bounce kernels were
            # measured to run up to 20% slower.
            host = {k: np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for k, v in arrays.items()}
            ptrs = {k: ctypes.c_void_p(v.ctypes.data) for k, v in host.items()}
            self._lib_stream.synchronize()
            entry = self.lib.emrt_set_frame_host
        desc = A.FrameDesc(int(frame_index), float(getattr(fr, "t", 0.0)), self.n_tx, self.n_rx, ptrs["xf"],
                           ptrs["ov"], ptrs["tx"], ptrs["txv"], ptrs["txo"], ptrs["rx"], ptrs["rxv"])
        self._check(entry(self.ctx, ctypes.byref(desc)))

    def step(self, discover: bool = True) -> int:
        self.generation += 1
        return self._check(self.lib.emrt_step(self.ctx, 1 if discover else 0))

    def step_rx(self, rx_ids: Sequence[int], rays_per_rx: int) -> int:
        """Discovery step launched from the given receivers (emrt_step_rx)."""
        self.generation += 1
        self._rev_host = np.ascontiguousarray(np.asarray(rx_ids, np.int32).reshape(-1))
        return self._check(self.lib.emrt_step_rx(self.ctx, self._rev_host.ctypes.data, len(self._rev_host),
                                                 int(rays_per_rx)))

    def sync(self) -> int:
        return self._check(self.lib.emrt_sync(self.ctx))

    # --------------------------------------------------------------- outputs
    def channels(self) -> Dict[str, torch.Tensor]:
        nf, nl, d = len(self.freqs), self.n_links, self.device
        out = {
            "H": torch.empty((nf, nl, 2), dtype=torch.float64, device=d),
            "P_coh": torch.empty((nf, nl), dtype=torch.float64, device=d),
            "P_inc": torch.empty((nf, nl), dtype=torch.float64, device=d),
            "tau_mean": torch.empty((nf, nl), dtype=torch.float64, device=d),
            "tau_rms": torch.empty((nf, nl), dtype=torch.float64, device=d),
            "fd_mean": torch.empty((nf, nl), dtype=torch.float64, device=d),
            "fd_rms": torch.empty((nf, nl), dtype=torch.float64, device=d),
            "n_paths": torch.empty((nl,), dtype=torch.int32, device=d),
            "flags": torch.empty((nl,), dtype=torch.int32, device=d),
        }
        v = A.ChannelView(*(_ptr(out[k]) for k in ("H", "P_coh", "P_inc", "tau_mean", "tau_rms", "fd_mean", "fd_rms",
                                                   "n_paths", "flags")))
        self._check(self.lib.emrt_read_channels(self.ctx, ctypes.byref(v)))
        out["H"] = torch.view_as_complex(out["H"])
        return out

    def paths(self, cap: Optional[int] = None) -> Dict[str, torch.Tensor]:
        cap = int(cap or self.cfg.path_cap_per_link)
        nf, nl, d = len(self.freqs), self.n_links, self.device
        out = {
            "key": torch.empty((nl, cap, 9), dtype=torch.int32, device=d),
            "tri_ids": torch.empty((nl, cap, 5), dtype=torch.int32, device=d),
            "a": torch.empty((nl, cap, nf, 2), dtype=torch.float64, device=d),
            "tau": torch.empty((nl, cap), dtype=torch.float64, device=d),
            "fd": torch.empty((nl, cap, nf), dtype=torch.float64, device=d),
            "angles": torch.empty((nl, cap, 4), dtype=torch.float32, device=d),
            "count": torch.empty((nl,), dtype=torch.int32, device=d),
        }
        v = A.PathView(cap, *(_ptr(out[k]) for k in ("key", "tri_ids", "a", "tau", "fd", "angles", "count")))
        st = self._check(self.lib.emrt_read_paths(self.ctx, ctypes.byref(v)))
        out["truncated"] = st == A.EMRT_W_PATHS_TRUNCATED
        out["a"] = torch.view_as_complex(out["a"])
        return out

    def flat_paths(self, cap: Optional[int] = None) -> Dict[str, np.ndarray]:
        """All paths of the last step as flat host arrays (keys in link, key order)."""
        p = self.paths(cap)
        cnt = p["count"].cpu().numpy()
        mask = np.arange(p["key"].shape[1])[None, :] < cnt[:, None]
        res = {k: p[k].cpu().numpy()[mask] for k in ("key", "tri_ids", "a", "tau", "fd", "angles")}
        res["truncated"] = p["truncated"]
        return res

    def backward(self, dL_dH: Optional[torch.Tensor] = None,
                 dL_dP: Optional[torch.Tensor] = None) -> Dict[str, torch.Tensor]:
        """Adjoint of the last step (emrt_backward).  dL_dH complex [n_freq,
        n_links] (dL/dRe H + j dL/dIm H), dL_dP real [n_freq, n_links]
        (dL/dP_coh); returns grad_eps complex [n_materials], grad_tx_pos
        [n_tx, 3] and grad_tx_orient [n_tx, 2]."""
        nf, nl, d = len(self.freqs), self.n_links, self.device
        gh = None
        if dL_dH is not None:
            gh = torch.view_as_real(dL_dH.to(device=d, dtype=torch.complex128).reshape(nf, nl).contiguous()).contiguous()
        gp = None if dL_dP is None else dL_dP.to(device=d, dtype=torch.float64).reshape(nf, nl).contiguous()
        m = len(self._mat_host)
        out = {
            "grad_eps": torch.empty((m, 2), dtype=torch.float64, device=d),
            "grad_tx_pos": torch.empty((self.n_tx, 3), dtype=torch.float64, device=d),
            "grad_tx_orient": torch.empty((self.n_tx, 2), dtype=torch.float64, device=d),
        }
        self._check(self.lib.emrt_backward(self.ctx, _ptr(gh), _ptr(gp), _ptr(out["grad_eps"]),
                                           _ptr(out["grad_tx_pos"]), _ptr(out["grad_tx_orient"])))
        self._check(self.lib.emrt_sync(self.ctx))
        self._bw_refs = (gh, gp)
        out["grad_eps"] = torch.view_as_complex(out["grad_eps"])
        return out

    def coherence(self, R: float = 0.5) -> Dict[str, object]:
        """Coherence statistics after the last step (emrt_read_coherence):
        tc [n_freq, n_links] (Eq (2)), corr [n_freq, n_links, 4] (Eq (1) at
        lags 1..4 frames), trigger [n_links], min_tc, n_triggered."""
        nf, nl, d = len(self.freqs), self.n_links, self.device
        out = {
            "tc": torch.empty((nf, nl), dtype=torch.float64, device=d),
            "corr": torch.empty((nf, nl, A.CORR_LAGS), dtype=torch.float64, device=d),
            "trigger": torch.empty((nl,), dtype=torch.int32, device=d),
        }
        v = A.CoherenceView(_ptr(out["tc"]), _ptr(out["corr"]), _ptr(out["trigger"]))
        mt, nt = ctypes.c_double(), ctypes.c_int64()
        self._check(self.lib.emrt_read_coherence(self.ctx, float(R), ctypes.byref(v), ctypes.byref(mt),
                                                 ctypes.byref(nt)))
        out["min_tc"] = mt.value
        out["n_triggered"] = nt.value
        return out

    def coherence_reset(self) -> None:
        self._check(self.lib.emrt_coherence_reset(self.ctx))

    def debug_rays(self, tx: int, ray_ids) -> np.ndarray:
        ids = _dev(ray_ids, torch.int32, self.device)
        out = torch.empty((len(ids), int(self.cfg.max_reflections) + 1), dtype=torch.int32, device=self.device)
        self._check(self.lib.emrt_debug_ray_records(self.ctx, int(tx), _ptr(ids), len(ids), _ptr(out)))
        return out.cpu().numpy()

    def debug_select_rays(self, tx: int, ray_ids) -> None:
        """Mark launch directions ray_ids of transmitter tx for the capture log
        of later transmitter-side discovery steps (an empty list clears all)."""
        ids = _dev(np.asarray(ray_ids, np.int32).reshape(-1), torch.int32, self.device)
        self._check(self.lib.emrt_debug_select_rays(self.ctx, int(tx), _ptr(ids) if len(ids) else None, len(ids)))

    def debug_ray_captures(self) -> np.ndarray:
        """Capture log of the last transmitter-side discovery step: rows (tx,
        launch direction, bounce, kind 0 receiver / 1 edge, receiver or edge
        id).  Raises when rows were dropped."""
        out = torch.empty((A.CAPTURE_LOG_ROWS, 5), dtype=torch.int32, device=self.device)
        n = ctypes.c_int64()
        st = self._check(self.lib.emrt_debug_ray_captures(self.ctx, _ptr(out), A.CAPTURE_LOG_ROWS, ctypes.byref(n)))
        if st == A.EMRT_W_PATHS_TRUNCATED:
            raise EmrtError(st, "capture log overflow: mark fewer rays")
        return out[: n.value].cpu().numpy()

    def cache_export(self) -> np.ndarray:
        n = ctypes.c_int64()
        self._check(self.lib.emrt_cache_size(self.ctx, ctypes.byref(n)))
        buf = torch.empty((max(n.value, 1), 9), dtype=torch.int32, device=self.device)
        self._check(self.lib.emrt_cache_export(self.ctx, _ptr(buf), n.value, ctypes.byref(n)))
        return buf[: n.value].cpu().numpy()

    def cache_import(self, keys) -> None:
        k = _dev(np.asarray(keys, np.int32).reshape(-1, 9), torch.int32, self.device)
        self._check(self.lib.emrt_cache_import(self.ctx, _ptr(k), len(k)))

    def set_instrumentation(self, stats: bool = False, timing: bool = False) -> None:
        self._check(self.lib.emrt_set_instrumentation(self.ctx, int(stats), int(timing)))

    def stats(self) -> Dict[str, object]:
        s = A.Stats()
        self._check(self.lib.emrt_read_stats(self.ctx, ctypes.byref(s)))
        return {f: (list(getattr(s, f)) if f == "rays_per_bounce" else getattr(s, f)) for f, _ in A.Stats._fields_}


class Batch:
    """Batched stepping of several Tracers (emrt_batch): the members' bounces
    run as one persistent launch per bounce level and the step is replayed
    from a HIP graph.  Frames are set and results read on the member
    Tracers; ``step`` replaces their individual ``step``."""

    def __init__(self, tracers: Sequence[Tracer], use_graph: bool = True, n_streams: int = 4, grid: int = 2048,
                 chunk: int = 64):
        self.lib = A.load()
        self.tracers = list(tracers)
        n = len(self.tracers)
        arr = (ctypes.c_void_p * n)(*[t.ctx.value for t in self.tracers])
        b = ctypes.c_void_p()
        st = self.lib.emrt_batch_create(arr, n, ctypes.byref(b))
        if st < 0:
            raise EmrtError(st, A.load().emrt_status_string(st).decode())
        self.b = b
        nbytes = ctypes.c_size_t()
        self._check(self.lib.emrt_batch_workspace_size(self.b, ctypes.byref(nbytes)))
        dev = self.tracers[0].device
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=dev)
        # graph capture needs a stream other than the device's default stream
        self.stream = torch.cuda.Stream(device=dev)
        torch.cuda.current_stream(dev).synchronize()
        self._check(self.lib.emrt_batch_set_stream(self.b, ctypes.c_void_p(self.stream.cuda_stream)))
        for t in self.tracers:
            t._lib_stream = self.stream
        self._check(self.lib.emrt_batch_bind_workspace(self.b, ctypes.c_void_p(_ptr(self.workspace)), nbytes.value))
        self.use_graph = bool(use_graph)
        self.set_options(use_graph, n_streams, grid, chunk)

    def _check(self, st: int) -> int:
        if st < 0:
            buf = ctypes.create_string_buffer(512)
            self.lib.emrt_batch_last_error(self.b, buf, 512)
            raise EmrtError(st, buf.value.decode() or A.load().emrt_status_string(st).decode())
        return st

    def set_options(self, use_graph: bool = True, n_streams: int = 4, grid: int = 2048, chunk: int = 64) -> None:
        self.use_graph = bool(use_graph)
        self.options = dict(n_streams=int(n_streams), grid=int(grid), chunk=int(chunk))
        self._check(self.lib.emrt_batch_set_options(self.b, int(use_graph), int(n_streams), int(grid), int(chunk)))

    def step(self, discover: bool = True) -> int:
        for t in self.tracers:
            t.generation += 1
        return self._check(self.lib.emrt_batch_step(self.b, 1 if discover else 0))

    def tune_key(self) -> str:
        """Autotuning cache key: the GPU architecture and size buckets (powers
        of two of the members' primary rays and of the member count)."""
        dev = self.tracers[0].device
        arch = torch.cuda.get_device_properties(dev).gcnArchName.split(":")[0]
        rays = sum(int(t.n_tx) * int(t.cfg.rays_per_tx) for t in self.tracers)
        return f"{arch}|rays_2^{round(math.log2(max(rays, 1)))}|scenes_2^{round(math.log2(len(self.tracers)))}"

    def autotune(self, repeats: int = 3, cache: Optional[str] = None) -> Dict[str, object]:
        """Launch shape (grid, streams, chunk) from the JSON cache file `cache`
        when it holds this batch's key, else timed by emrt_batch_autotune
        (`repeats` timed steps per combination, median) and stored there."""
        key = self.tune_key()
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        if key in table:
            o = table[key]
            self.set_options(self.use_graph, o["streams"], o["grid"], o["chunk"])
            return dict(o, key=key, from_cache=True)
        g, s, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.emrt_batch_autotune(self.b, int(repeats), ctypes.byref(g), ctypes.byref(s),
                                                 ctypes.byref(c)))
        self.options = dict(n_streams=s.value, grid=g.value, chunk=c.value)
        o = {"grid": g.value, "streams": s.value, "chunk": c.value, "repeats": int(repeats)}
        if cache:
            table[key] = o
            d = os.path.dirname(os.path.abspath(cache))
            os.makedirs(d, exist_ok=True)
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return dict(o, key=key, from_cache=False)

    def sync(self) -> int:
        return self._check(self.lib.emrt_batch_sync(self.b))

    def close(self) -> None:
        if getattr(self, "b", None):
            torch.cuda.synchronize(self.tracers[0].device)
            self.lib.emrt_batch_destroy(self.b)
            self.b = None
            for t in self.tracers:  # the members work on their own streams again
                t._lib_stream = t.stream

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
