"""Python binding of libmrf: torch tensors in, torch tensors out.

PyTorch provides device memory and streams only; every step of the method
runs in libmrf's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Optional

import numpy as np
import torch

from . import _lib as L


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Context:
    def __init__(self, device: int = 0):
        self._lib = L.load()
        h = C.c_void_p()
        L.check(self._lib.mrf_context_create(int(device), C.byref(h)))
        self.handle = h
        self.device = torch.device("cuda", int(device))

    def close(self):
        if self.handle:
            self._lib.mrf_context_destroy(self.handle)
            self.handle = None

    def profile(self, enable: bool = True):
        L.check(self._lib.mrf_profile_enable(self.handle, int(bool(enable))))

    def profile_read(self, kernel: str, reset: bool = True):
        """(total ms, launches) of a named kernel since the last reset."""
        ms = C.c_double()
        n = C.c_int64()
        L.check(self._lib.mrf_profile_read(self.handle, kernel.encode(), int(bool(reset)),
                                           C.byref(ms), C.byref(n)))
        return float(ms.value), int(n.value)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sequence:
    """A sequence resident in libmrf (host description + device copy)."""

    def __init__(self, ctx: Context, seq):
        self.ctx = ctx
        self.seq = seq
        self._keep = [np.ascontiguousarray(x, np.float64) for x in
                      (seq.fa_deg, seq.phase_deg, seq.tr_ms, seq.te_ms)]
        d = L.SequenceDesc(len(self._keep[0]), *[_dp(x) for x in self._keep],
                           int(seq.inversion), float(seq.ti_ms), int(getattr(seq, "smooth", 0)))
        h = C.c_void_p()
        L.check(ctx._lib.mrf_sequence_create(ctx.handle, C.byref(d), C.byref(h)))
        self.handle = h
        self.n = len(self._keep[0])

    def close(self):
        if self.handle:
            self.ctx._lib.mrf_sequence_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GridArg:
    """ctypes view of an inputs.Grid (keeps the numpy buffers alive)."""

    def __init__(self, grid):
        self.grid = grid
        self._keep = [np.ascontiguousarray(a, np.float64) for a in
                      (grid.t1_ms, grid.t2_ms, grid.df_hz, grid.b1)]
        ax = [L.Axis(len(a), _dp(a) if len(a) else None) for a in self._keep]
        self.desc = L.GridDesc(*ax)

    @property
    def ptr(self):
        return C.byref(self.desc)


@dataclasses.dataclass
class Dictionary:
    """A simulated dictionary in HBM.

    f32 : re, im float32 [n_tr, ld] (planar, time-major)
    bf16: packed bfloat16 blocks viewed as int16 [n_tr/4, ld, 4, 2]
    f32rows: entry-major complex64 rows, re float32 [n_entries, ld, 2] (ld even
          and >= n_tr; the layout the resident-dictionary ZOOM reads)
    norm: float64 [n_entries] raw norms (None when the entries are unit-norm)
    """
    dtype: str
    n_tr: int
    n_entries: int
    ld: int
    re: torch.Tensor
    im: Optional[torch.Tensor]
    norm: Optional[torch.Tensor]
    entry_base: int = 0

    def view(self, n_tr: Optional[int] = None) -> L.DictView:
        n = self.n_tr if n_tr is None else int(n_tr)
        return L.DictView(_DTYPES[self.dtype], n, self.n_entries,
                          self.ld, self.re.data_ptr(),
                          self.im.data_ptr() if self.im is not None else None,
                          self.norm.data_ptr() if self.norm is not None else None,
                          self.entry_base)

    @property
    def nbytes(self) -> int:
        b = self.re.numel() * self.re.element_size()
        if self.im is not None:
            b += self.im.numel() * self.im.element_size()
        return b


def _round_up(x: int, m: int) -> int:
    return (x + m - 1) // m * m


_DTYPES = {"f32": L.MRF_F32, "bf16": L.MRF_BF16, "f32rows": L.MRF_F32_ROWS}


def alloc_dictionary(n_tr: int, n_entries: int, dtype: str = "f32", device="cuda",
                     ld: Optional[int] = None, with_norm: bool = True) -> Dictionary:
    if dtype == "f32rows":
        ld = _round_up(n_tr, 16) if ld is None else int(ld)  # 128-byte aligned rows
        re = torch.empty((max(n_entries, 1), ld, 2), dtype=torch.float32, device=device)
        norm = torch.empty(n_entries, dtype=torch.float64, device=device) if with_norm else None
        return Dictionary(dtype, n_tr, n_entries, ld, re, None, norm)
    ld = _round_up(max(n_entries, 1), 256) if ld is None else int(ld)
    if dtype == "f32":
        re = torch.empty((n_tr, ld), dtype=torch.float32, device=device)
        im = torch.empty((n_tr, ld), dtype=torch.float32, device=device)
    elif dtype == "bf16":
        if n_tr % 4:
            raise ValueError("BF16 dictionaries need n_tr % 4 == 0")
        re = torch.empty((n_tr // 4, ld, 4, 2), dtype=torch.int16, device=device)
        im = None
    else:
        raise ValueError(dtype)
    norm = torch.empty(n_entries, dtype=torch.float64, device=device) if with_norm else None
    return Dictionary(dtype, n_tr, n_entries, ld, re, im, norm)


def simulate_dictionary(ctx: Context, seq: Sequence, grid, n_tr: Optional[int] = None,
                        dtype: str = "f32", entry_begin: int = 0,
                        entry_count: Optional[int] = None, unit_norm: bool = False,
                        out: Optional[Dictionary] = None, stream=None) -> Dictionary:
    n_tr = seq.n if n_tr is None else int(n_tr)
    g = grid if isinstance(grid, GridArg) else GridArg(grid)
    count = g.grid.size - entry_begin if entry_count is None else int(entry_count)
    d = out if out is not None else alloc_dictionary(n_tr, count, dtype, ctx.device,
                                                     with_norm=True)
    d.entry_base = int(entry_begin)
    L.check(ctx._lib.mrf_simulate_dictionary(
        ctx.handle, seq.handle, g.ptr, n_tr, int(entry_begin), count,
        _DTYPES[d.dtype], d.re.data_ptr(),
        d.im.data_ptr() if d.im is not None else None, d.ld,
        d.norm.data_ptr() if d.norm is not None else None, int(bool(unit_norm)),
        _stream_ptr(stream)))
    if unit_norm:
        d_norm_raw = d.norm
        d.norm = None
        d.raw_norm = d_norm_raw  # type: ignore[attr-defined]
    return d


def simulate_dictionary_pair(ctx: Context, seq: Sequence, grid, n_tr: Optional[int] = None,
                             entry_begin: int = 0, entry_count: Optional[int] = None,
                             out: Optional[tuple] = None, stream=None) -> tuple:
    """The FP32 planar and the BF16 dictionary of the same entries (raw
    values, with their norms) from one simulation pass: (d32, d16), as
    simulate_dictionary gives them for dtype "f32" and "bf16"."""
    n_tr = seq.n if n_tr is None else int(n_tr)
    g = grid if isinstance(grid, GridArg) else GridArg(grid)
    count = g.grid.size - entry_begin if entry_count is None else int(entry_count)
    if out is not None:
        d32, d16 = out
        if d32.ld != d16.ld:
            raise ValueError("the two dictionaries must share ld")
    else:
        d32 = alloc_dictionary(n_tr, count, "f32", ctx.device, with_norm=True)
        d16 = alloc_dictionary(n_tr, count, "bf16", ctx.device, with_norm=True)
    for d in (d32, d16):
        d.entry_base = int(entry_begin)
    L.check(ctx._lib.mrf_simulate_dictionary_pair(
        ctx.handle, seq.handle, g.ptr, n_tr, int(entry_begin), count, d32.re.data_ptr(),
        d32.im.data_ptr(), d16.re.data_ptr(), d32.ld,
        d32.norm.data_ptr() if d32.norm is not None else None,
        d16.norm.data_ptr() if d16.norm is not None else None, _stream_ptr(stream)))
    return d32, d16


def cc_map(ctx: Context, seq: Sequence, grid, vox: torch.Tensor, n_tr: Optional[int] = None,
           entry_begin: int = 0, entry_count: Optional[int] = None,
           out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """CC of Eq. 1 between each fingerprint (complex64 cuda [n_vox, >= n_tr])
    and every entry of [entry_begin, entry_begin + entry_count) of the grid,
    simulated on the fly (Experiment 1). Returns float32 cuda [n_vox, count]."""
    if vox.dtype != torch.complex64 or not vox.is_cuda:
        raise ValueError("vox must be a complex64 CUDA tensor")
    if vox.dim() == 1:
        vox = vox[None]
    if vox.stride(1) != 1:
        raise ValueError("vox rows must be contiguous")
    n_tr = seq.n if n_tr is None else int(n_tr)
    g = grid if isinstance(grid, GridArg) else GridArg(grid)
    count = g.grid.size - entry_begin if entry_count is None else int(entry_count)
    n_vox = vox.shape[0]
    if out is None:
        out = torch.empty((n_vox, count), dtype=torch.float32, device=ctx.device)
    if out.dtype != torch.float32 or out.dim() != 2 or out.stride(1) != 1 or \
            out.shape[0] < n_vox or out.shape[1] < count:
        raise ValueError("out must be float32 [>= n_vox, >= count] with contiguous rows")
    L.check(ctx._lib.mrf_cc_map(ctx.handle, seq.handle, g.ptr, n_tr, vox.data_ptr(), n_vox,
                                vox.stride(0), int(entry_begin), count, out.data_ptr(),
                                out.stride(0), _stream_ptr(stream)))
    return out


def simulate_signals(ctx: Context, seq: Sequence, params: torch.Tensor,
                     n_tr: Optional[int] = None, stream=None) -> torch.Tensor:
    """params: float64 cuda [count, 4] (T1, T2, df, B1) -> complex64 [count, n_tr]."""
    n_tr = seq.n if n_tr is None else int(n_tr)
    params = params.to(device=ctx.device, dtype=torch.float64).contiguous()
    out = torch.empty((params.shape[0], n_tr), dtype=torch.complex64, device=ctx.device)
    L.check(ctx._lib.mrf_simulate_signals(ctx.handle, seq.handle, n_tr, params.data_ptr(),
                                          params.shape[0], out.data_ptr(), n_tr,
                                          _stream_ptr(stream)))
    return out


def smooth_signals(ctx: Context, x: torch.Tensor, taps: int, out: Optional[torch.Tensor] = None,
                   seq: Optional[Sequence] = None, stream=None) -> torch.Tensor:
    """Temporal smoothing of complex64 cuda signals [n_sig, n_tr] along the
    readouts (taps 3 or 5; 0 or 1 copy), in the frame demodulated by seq's RF
    phases (None: zero phases). out=None returns a new tensor; out=x smooths
    in place."""
    if x.dtype != torch.complex64 or x.dim() != 2 or x.stride(1) != 1:
        raise ValueError("x must be complex64 [n_sig, n_tr] with unit stride along readouts")
    if out is None:
        out = torch.empty_like(x, memory_format=torch.contiguous_format)
    if out.dtype != torch.complex64 or out.shape != x.shape or out.stride(1) != 1:
        raise ValueError("out must be complex64 of x's shape with unit readout stride")
    L.check(ctx._lib.mrf_smooth_signals(ctx.handle, seq.handle if seq is not None else None,
                                        x.data_ptr(), x.stride(0), out.data_ptr(),
                                        out.stride(0), x.shape[0], x.shape[1], int(taps),
                                        _stream_ptr(stream)))
    return out


def match_workspace_bytes(ctx: Context, d: Dictionary, n_vox: int, top_k: int,
                          n_tr: Optional[int] = None) -> int:
    v = d.view(n_tr)
    b = C.c_size_t()
    L.check(ctx._lib.mrf_match_workspace(ctx.handle, C.byref(v), int(n_vox), int(top_k),
                                         C.byref(b)))
    return int(b.value)


class Workspace:
    """A reusable device byte buffer (grown on demand)."""

    def __init__(self, device):
        self.device = device
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self.buf


def _result_tensors(n_vox: int, device, with_nsim=False):
    return dict(idx=torch.empty(n_vox, dtype=torch.int64, device=device),
                cc=torch.empty(n_vox, dtype=torch.float32, device=device),
                margin=torch.empty(n_vox, dtype=torch.float32, device=device),
                pd_re=torch.empty(n_vox, dtype=torch.float32, device=device),
                pd_im=torch.empty(n_vox, dtype=torch.float32, device=device),
                **({"n_sim": torch.empty(n_vox, dtype=torch.int32, device=device)}
                   if with_nsim else {}))


def _result_view(r: dict) -> L.ResultView:
    p = lambda k: r[k].data_ptr() if k in r and r[k] is not None else None
    return L.ResultView(p("idx"), p("cc"), p("margin"), p("pd_re"), p("pd_im"), p("n_sim"))


def match_bruteforce(ctx: Context, d: Dictionary, vox: torch.Tensor, top_k: int = 1,
                     seq: Optional[Sequence] = None, grid=None, n_tr: Optional[int] = None,
                     workspace: Optional[Workspace] = None, with_topk: bool = False,
                     out: Optional[dict] = None, stream=None) -> dict:
    """vox: complex64 cuda [n_vox, >= n_tr]. Returns a dict of device tensors."""
    if vox.dtype != torch.complex64 or not vox.is_cuda:
        raise ValueError("vox must be a complex64 CUDA tensor")
    if vox.stride(1) != 1:
        raise ValueError("vox rows must be contiguous")
    n_vox = vox.shape[0]
    v = d.view(n_tr)
    ws = workspace if workspace is not None else Workspace(ctx.device)
    nb = match_workspace_bytes(ctx, d, n_vox, top_k, n_tr)
    buf = ws.get(nb)
    r = out if out is not None else _result_tensors(n_vox, ctx.device)
    tk_i = tk_c = None
    if with_topk:
        tk_i = torch.empty((n_vox, top_k), dtype=torch.int64, device=ctx.device)
        tk_c = torch.empty((n_vox, top_k), dtype=torch.float32, device=ctx.device)
        r["topk_idx"], r["topk_cc"] = tk_i, tk_c
    g = None
    if grid is not None:
        g = grid if isinstance(grid, GridArg) else GridArg(grid)
        r["_grid"] = g
    L.check(ctx._lib.mrf_match_bruteforce(
        ctx.handle, C.byref(v), vox.data_ptr(), n_vox, vox.stride(0), int(top_k),
        seq.handle if seq is not None else None, g.ptr if g is not None else None,
        _result_view(r), tk_i.data_ptr() if tk_i is not None else None,
        tk_c.data_ptr() if tk_c is not None else None, buf.data_ptr(), buf.numel(),
        _stream_ptr(stream)))
    return r


def match_bruteforce_noalloc(ctx: Context, d: Dictionary, vox: torch.Tensor, top_k: int = 1,
                             n_tr: Optional[int] = None, with_topk: bool = False,
                             out: Optional[dict] = None, stream=None) -> dict:
    """FP32 brute force through the allocation-free entry point (workspace in
    the library's static device array). Outputs as match_bruteforce; pass
    `out` (and preallocated topk tensors in it) to allocate nothing here."""
    if vox.dtype != torch.complex64 or not vox.is_cuda:
        raise ValueError("vox must be a complex64 CUDA tensor")
    if vox.stride(1) != 1:
        raise ValueError("vox rows must be contiguous")
    n_vox = vox.shape[0]
    v = d.view(n_tr)
    r = out if out is not None else _result_tensors(n_vox, ctx.device)
    if with_topk and "topk_idx" not in r:
        r["topk_idx"] = torch.empty((n_vox, top_k), dtype=torch.int64, device=ctx.device)
        r["topk_cc"] = torch.empty((n_vox, top_k), dtype=torch.float32, device=ctx.device)
    tk_i, tk_c = (r.get("topk_idx"), r.get("topk_cc")) if with_topk else (None, None)
    L.check(ctx._lib.mrf_match_bruteforce_noalloc(
        ctx.handle, C.byref(v), vox.data_ptr(), n_vox, vox.stride(0), int(top_k),
        _result_view(r), tk_i.data_ptr() if tk_i is not None else None,
        tk_c.data_ptr() if tk_c is not None else None, _stream_ptr(stream)))
    return r


# ---------------------------------------------------------------- ZOOM -----

STAGE_KINDS = {"scan_stride": 0, "scan_window": 1, "scan_hops": 2, "zoom1": 3, "zoom2": 4}


def schedule_to_dict(s: "L.ZoomSchedule") -> dict:
    st = lambda x: dict(kind=x.kind, axis0=x.axis0, axis1=x.axis1, step0=x.step0,
                        step1=x.step1, window=x.window, hop=x.hop, objective=x.objective)
    return dict(stages=[st(s.stages[i]) for i in range(s.n_stages)],
                outer=[st(s.outer[i]) for i in range(s.n_outer)], outer_max=s.outer_max,
                starts=[list(s.starts[i]) for i in range(s.n_starts)], pruned=s.pruned,
                prior_half=list(s.prior_half))


def schedule_from_dict(d: dict) -> "L.ZoomSchedule":
    s = L.ZoomSchedule()
    if len(d["stages"]) > L.ZOOM_MAX_STAGES or len(d.get("outer", [])) > L.ZOOM_MAX_STAGES:
        raise ValueError("too many stages")
    mk = lambda x: L.ZoomStage(x["kind"], x["axis0"], x.get("axis1", 0), x.get("step0", 0),
                               x.get("step1", 0), x.get("window", 0), x.get("hop", 0.0),
                               x.get("objective", L.OBJ_CC))
    s.n_stages = len(d["stages"])
    for i, x in enumerate(d["stages"]):
        s.stages[i] = mk(x)
    s.n_outer = len(d.get("outer", []))
    for i, x in enumerate(d.get("outer", [])):
        s.outer[i] = mk(x)
    s.outer_max = int(d.get("outer_max", 0))
    starts = d.get("starts", [[0, 0, 0, 0]])
    s.n_starts = len(starts)
    for i, st in enumerate(starts):
        for a in range(4):
            s.starts[i][a] = int(st[a])
    s.pruned = int(d.get("pruned", 0))
    for a, h in enumerate(d.get("prior_half", [-1, -1, -1, -1])):
        s.prior_half[a] = int(h)
    return s


def schedule_paper(ctx: Context, seq: Sequence, grid) -> dict:
    g = grid if isinstance(grid, GridArg) else GridArg(grid)
    s = L.ZoomSchedule()
    L.check(ctx._lib.mrf_zoom_schedule_paper(g.ptr, seq.handle, C.byref(s)))
    return schedule_to_dict(s)


def schedule_multistart(ctx: Context, seq: Sequence, grid, n_t1: int = 4, n_t2: int = 4,
                        outer_max: int = 8) -> dict:
    """The paper's stages from an n_t1 x n_t2 lattice of starts with an outer
    refinement round (see mrf_zoom_schedule_multistart)."""
    g = grid if isinstance(grid, GridArg) else GridArg(grid)
    s = L.ZoomSchedule()
    L.check(ctx._lib.mrf_zoom_schedule_multistart(g.ptr, seq.handle, int(n_t1), int(n_t2),
                                                  int(outer_max), C.byref(s)))
    return schedule_to_dict(s)


def schedule_finest_objective(sched: dict, objective: int = 1) -> dict:
    """A copy of the schedule with every finest-resolution (unit-step) stage
    scored by `objective` (libmrf mrf_zoom_schedule_finest_objective; 1: the
    distance of the non-normalised fingerprint)."""
    s = schedule_from_dict(sched)
    L.check(L.load().mrf_zoom_schedule_finest_objective(C.byref(s), int(objective)))
    return schedule_to_dict(s)


def schedule_local(grid, outer_max: int = 8) -> dict:
    """Unit-step local refinement schedule (see mrf_zoom_schedule_local)."""
    lib = L.load()
    g = grid if isinstance(grid, GridArg) else GridArg(grid)
    s = L.ZoomSchedule()
    L.check(lib.mrf_zoom_schedule_local(g.ptr, int(outer_max), C.byref(s)))
    return schedule_to_dict(s)


def grid_indices(grid, idx) -> np.ndarray:
    """Flat grid indices -> int32 [n, 4] per-axis indices (the init_idx layout)."""
    gr = grid.grid if isinstance(grid, GridArg) else grid
    k = np.asarray(idx, dtype=np.int64)
    n4 = max(len(gr.b1), 1)
    n3, n2 = len(gr.df_hz), len(gr.t2_ms)
    i4 = k % n4
    k = k // n4
    i3 = k % n3
    k = k // n3
    i2 = k % n2
    i1 = k // n2
    return np.stack([i1, i2, i3, i4], axis=1).astype(np.int32)


def zoom_search(ctx: Context, seq: Sequence, grid, vox: torch.Tensor, sched: Optional[dict] = None,
                n_tr: Optional[int] = None, init: Optional[torch.Tensor] = None,
                workspace: Optional[Workspace] = None, out: Optional[dict] = None,
                stream=None, start: Optional[torch.Tensor] = None) -> dict:
    """MRF-ZOOM per voxel. vox: complex64 cuda [n_vox, >= n_tr]; init: int32 cuda
    [n_vox, 4] prior centres, or start: int64 cuda [n_vox] prior centres as flat
    grid indices. Returns idx, cc, margin (min decision margin), pd_re, pd_im,
    n_sim."""
    if vox.dtype != torch.complex64 or not vox.is_cuda or vox.stride(1) != 1:
        raise ValueError("vox must be a complex64 CUDA tensor with contiguous rows")
    n_tr = seq.n if n_tr is None else int(n_tr)
    g = grid if isinstance(grid, GridArg) else GridArg(grid)
    sd = schedule_paper(ctx, seq, g) if sched is None else sched
    s = schedule_from_dict(sd)
    n_vox = vox.shape[0]
    nb = C.c_size_t()
    L.check(ctx._lib.mrf_zoom_workspace(ctx.handle, g.ptr, n_vox, n_tr, C.byref(nb)))
    ws = workspace if workspace is not None else Workspace(ctx.device)
    buf = ws.get(int(nb.value))
    r = out if out is not None else _result_tensors(n_vox, ctx.device, with_nsim=True)
    if start is not None:
        # prior centres as flat grid indices (e.g. a brute-force idx output)
        start = start.to(device=ctx.device, dtype=torch.int64).contiguous()
        r["_start"] = start
        L.check(ctx._lib.mrf_zoom_search_from(
            ctx.handle, seq.handle, g.ptr, C.byref(s), vox.data_ptr(), n_vox, vox.stride(0),
            n_tr, start.data_ptr(), _result_view(r), buf.data_ptr(), buf.numel(),
            _stream_ptr(stream)))
        return r
    if init is not None:
        init = init.to(device=ctx.device, dtype=torch.int32).contiguous()
        r["_init"] = init
    L.check(ctx._lib.mrf_zoom_search(
        ctx.handle, seq.handle, g.ptr, C.byref(s), vox.data_ptr(), n_vox, vox.stride(0), n_tr,
        init.data_ptr() if init is not None else None, _result_view(r), buf.data_ptr(),
        buf.numel(), _stream_ptr(stream)))
    return r


def zoom_search_ragged(ctx: Context, seq: Sequence, grid, vox: torch.Tensor,
                       vox_n_tr: torch.Tensor, sched: Optional[dict] = None,
                       workspace: Optional[Workspace] = None, out: Optional[dict] = None,
                       stream=None) -> dict:
    """MRF-ZOOM over voxels with their own readout counts (int32 cuda [n_vox],
    each <= vox.shape[1] and the sequence length) in one launch."""
    if vox.dtype != torch.complex64 or not vox.is_cuda or vox.stride(1) != 1:
        raise ValueError("vox must be a complex64 CUDA tensor with contiguous rows")
    vn = vox_n_tr.to(device=ctx.device, dtype=torch.int32).contiguous()
    n_tr = int(vn.max().item()) if vn.numel() else 1
    g = grid if isinstance(grid, GridArg) else GridArg(grid)
    s = schedule_from_dict(schedule_paper(ctx, seq, g) if sched is None else sched)
    n_vox = vox.shape[0]
    nb = C.c_size_t()
    L.check(ctx._lib.mrf_zoom_workspace(ctx.handle, g.ptr, n_vox, n_tr, C.byref(nb)))
    ws = workspace if workspace is not None else Workspace(ctx.device)
    buf = ws.get(int(nb.value))
    r = out if out is not None else _result_tensors(n_vox, ctx.device, with_nsim=True)
    r["_n_tr"] = vn
    L.check(ctx._lib.mrf_zoom_search_ragged(
        ctx.handle, seq.handle, g.ptr, C.byref(s), vox.data_ptr(), n_vox, vox.stride(0), n_tr,
        vn.data_ptr(), _result_view(r), buf.data_ptr(), buf.numel(), _stream_ptr(stream)))
    return r


def zoom_search_dict(ctx: Context, d: Dictionary, grid, vox: torch.Tensor, sched: dict,
                     n_tr: Optional[int] = None, init: Optional[torch.Tensor] = None,
                     workspace: Optional[Workspace] = None, out: Optional[dict] = None,
                     stream=None) -> dict:
    """MRF-ZOOM reading visited entries from a resident f32rows dictionary of
    the whole grid (mrf_zoom_search_dict). Outputs as zoom_search."""
    if vox.dtype != torch.complex64 or not vox.is_cuda or vox.stride(1) != 1:
        raise ValueError("vox must be a complex64 CUDA tensor with contiguous rows")
    if d.dtype != "f32rows":
        raise ValueError("the resident dictionary must be f32rows")
    n_tr = d.n_tr if n_tr is None else int(n_tr)
    g = grid if isinstance(grid, GridArg) else GridArg(grid)
    s = schedule_from_dict(sched)
    n_vox = vox.shape[0]
    nb = C.c_size_t()
    L.check(ctx._lib.mrf_zoom_workspace(ctx.handle, g.ptr, n_vox, n_tr, C.byref(nb)))
    ws = workspace if workspace is not None else Workspace(ctx.device)
    buf = ws.get(int(nb.value))
    r = out if out is not None else _result_tensors(n_vox, ctx.device, with_nsim=True)
    if init is not None:
        init = init.to(device=ctx.device, dtype=torch.int32).contiguous()
        r["_init"] = init
    v = d.view()  # the stored readout count; the search uses the first n_tr
    L.check(ctx._lib.mrf_zoom_search_dict(
        ctx.handle, C.byref(v), g.ptr, C.byref(s), vox.data_ptr(), n_vox, vox.stride(0), n_tr,
        init.data_ptr() if init is not None else None, _result_view(r), buf.data_ptr(),
        buf.numel(), _stream_ptr(stream)))
    return r


# ------------------------------------------------------------- serving -----

class Server:
    """Request loop over resident dictionaries (libmrf mrf_server_*).

    fake=True runs the scheduler against a host-simulated device (no GPU, no
    outputs written): requests then need only n_vox, not tensors."""

    def __init__(self, ctx: Optional[Context], budget_bytes: int, max_inflight: int = 64,
                 n_streams: int = 2, max_batch_vox: int = 0, fake: bool = False,
                 fake_ns_per_byte: float = 0.0, fake_fail_ticket: int = 0,
                 refine_bf16: bool = False, batch_window_ms: float = 0.0):
        self._lib = L.load()
        self.ctx = ctx
        cfg = L.ServerConfig(int(budget_bytes), int(max_inflight), int(n_streams),
                             int(max_batch_vox), int(bool(fake)), float(fake_ns_per_byte),
                             int(fake_fail_ticket), int(bool(refine_bf16)),
                             float(batch_window_ms))
        h = C.c_void_p()
        L.check(self._lib.mrf_server_create(ctx.handle if ctx is not None else None,
                                            C.byref(cfg), C.byref(h)))
        self.handle = h
        self.fake = bool(fake)
        self._keep = {}    # ticket -> tensors that must outlive the request
        self._grids = []

    def register(self, seq: Optional[Sequence], grid, dtype: str = "bf16", lengths=(1000,)) -> int:
        g = grid if isinstance(grid, GridArg) else GridArg(grid)
        self._grids.append(g)
        n = (C.c_int32 * len(lengths))(*[int(x) for x in lengths])
        slot = C.c_int32()
        L.check(self._lib.mrf_server_register(
            self.handle, seq.handle if seq is not None else None, g.ptr,
            L.MRF_F32 if dtype == "f32" else L.MRF_BF16, n, len(lengths), C.byref(slot)))
        return int(slot.value)

    def submit(self, mode: str, slot: int, n_tr: int, vox: Optional[torch.Tensor] = None,
               out: Optional[dict] = None, n_vox: Optional[int] = None) -> int:
        """mode 'brute' or 'zoom'. vox: complex64 cuda [n_vox, >= n_tr]; out: result
        tensors (see _result_tensors; created if None). Returns the ticket."""
        m = L.SERVE_BRUTE if mode == "brute" else L.SERVE_ZOOM
        if vox is not None:
            if vox.dtype != torch.complex64 or not vox.is_cuda or vox.stride(1) != 1:
                raise ValueError("vox must be a complex64 CUDA tensor with contiguous rows")
            nv = vox.shape[0]
            r = out if out is not None else _result_tensors(nv, vox.device, with_nsim=m == 1)
            req = L.Request(m, slot, n_tr, nv, vox.data_ptr(), vox.stride(0), _result_view(r))
        else:
            if not self.fake:
                raise ValueError("vox is required on a real device")
            nv, r = int(n_vox), None
            dummy = 1 << 12  # never dereferenced by the fake device
            req = L.Request(m, slot, n_tr, nv, dummy, n_tr, L.ResultView(dummy))
        t = C.c_uint64()
        L.check(self._lib.mrf_serve_submit(self.handle, C.byref(req), C.byref(t)))
        self._keep[int(t.value)] = (vox, r)
        return int(t.value)

    def result(self, ticket: int) -> Optional[dict]:
        return self._keep[ticket][1]

    def poll(self, ticket: int):
        """(state, t_submit_ms, t_start_ms, t_done_ms); raises MRFError for a failed request."""
        st, a, b, c = C.c_int32(), C.c_double(), C.c_double(), C.c_double()
        L.check(self._lib.mrf_serve_poll(self.handle, int(ticket), C.byref(st), C.byref(a),
                                         C.byref(b), C.byref(c)))
        state = L.REQ_STATES[st.value]
        return state, a.value, b.value, c.value

    def failure(self, ticket: int) -> str:
        self.poll(ticket)
        return self._lib.mrf_last_error().decode(errors="replace")

    def cancel(self, ticket: int):
        L.check(self._lib.mrf_serve_cancel(self.handle, int(ticket)))

    def stats(self) -> dict:
        s = L.ServerStats()
        L.check(self._lib.mrf_server_stats_read(self.handle, C.byref(s)))
        val = lambda x: list(x) if isinstance(x, C.Array) else x
        return {k: val(getattr(s, k)) for k, _ in L.ServerStats._fields_}

    def wait(self, tickets, timeout_s: float = 60.0, sleep_s: float = 0.0005):
        import time
        t_end = time.monotonic() + timeout_s
        pending = set(tickets)
        while pending:
            for t in list(pending):
                if self.poll(t)[0] in ("done", "failed", "cancelled"):
                    pending.discard(t)
            if pending:
                if time.monotonic() > t_end:
                    raise TimeoutError(f"{len(pending)} requests still pending")
                time.sleep(sleep_s)

    def close(self):
        if getattr(self, "handle", None):
            self._lib.mrf_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def prior_half_widths(grid, t1_ms=3000.0, t2_ms=800.0, df_hz=150.0, b1=0.3) -> list:
    """Neighbour-prior half widths in index steps for physical ranges (the
    Methods' Experiment 3 ranges by default; B1 +-0.3 for a B1 axis), as
    libmrf's mrf_zoom_schedule_prior converts them; -1 for an axis of one
    value."""
    lib = L.load()
    g = grid if isinstance(grid, GridArg) else GridArg(grid)
    half = (C.c_double * 4)(float(t1_ms), float(t2_ms), float(df_hz), float(b1))
    s = L.ZoomSchedule()
    L.check(lib.mrf_zoom_schedule_prior(g.ptr, half, C.byref(s)))
    return [int(s.prior_half[a]) for a in range(4)]


def schedule_with_prior(sched: dict, grid, half=None) -> dict:
    """A copy of `sched` whose prior_half is set by mrf_zoom_schedule_prior
    from physical half widths (T1 ms, T2 ms, df Hz, B1); None: the paper's
    Experiment 3 ranges."""
    lib = L.load()
    g = grid if isinstance(grid, GridArg) else GridArg(grid)
    s = schedule_from_dict(sched)
    h = None if half is None else (C.c_double * 4)(*[float(x) for x in half])
    L.check(lib.mrf_zoom_schedule_prior(g.ptr, h, C.byref(s)))
    return schedule_to_dict(s)


def zoom_search_lattice(ctx: Context, seq: Sequence, grid, vox: torch.Tensor, width: int,
                        height: int, n_slices: int, sched: Optional[dict] = None,
                        stride: int = 4, n_tr: Optional[int] = None,
                        workspace: Optional[Workspace] = None, out: Optional[dict] = None,
                        stream=None) -> dict:
    """MRF-ZOOM over a volume with the two-pass lattice neighbour prior
    (mrf_zoom_search_lattice). vox: complex64 cuda [n_slices*height*width,
    >= n_tr], slice-major raster order. sched['prior_half'] sets the pass-2
    ranges (see prior_half_widths)."""
    if vox.dtype != torch.complex64 or not vox.is_cuda or vox.stride(1) != 1:
        raise ValueError("vox must be a complex64 CUDA tensor with contiguous rows")
    n_tr = seq.n if n_tr is None else int(n_tr)
    g = grid if isinstance(grid, GridArg) else GridArg(grid)
    sd = schedule_paper(ctx, seq, g) if sched is None else sched
    s = schedule_from_dict(sd)
    n_vox = vox.shape[0]
    if n_vox != width * height * n_slices:
        raise ValueError("vox rows must equal width * height * n_slices")
    nb = C.c_size_t()
    L.check(ctx._lib.mrf_zoom_workspace(ctx.handle, g.ptr, n_vox, n_tr, C.byref(nb)))
    ws = workspace if workspace is not None else Workspace(ctx.device)
    buf = ws.get(int(nb.value))
    r = out if out is not None else _result_tensors(n_vox, ctx.device, with_nsim=True)
    L.check(ctx._lib.mrf_zoom_search_lattice(
        ctx.handle, seq.handle, g.ptr, C.byref(s), vox.data_ptr(), int(width), int(height),
        int(n_slices), vox.stride(0), n_tr, int(stride), _result_view(r), buf.data_ptr(),
        buf.numel(), _stream_ptr(stream)))
    return r


# ---- device peak probes (measurement aids, not steps of the method) ----

def probe_mfma(ctx: Context, dtype: str, iters: int, out: torch.Tensor, stream=None) -> float:
    """MFMA-only loop (libmrf mrf_probe_mfma) writing each lane's accumulator
    sum into out (float32 cuda, length a multiple of 256: one workgroup per
    256). Returns the flops the launch performs; it does not wait."""
    if out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 CUDA tensor")
    fl = C.c_double()
    L.check(ctx._lib.mrf_probe_mfma(ctx.handle, L.MRF_F32 if dtype == "f32" else L.MRF_BF16,
                                    int(iters), out.data_ptr(), out.numel(), C.byref(fl),
                                    _stream_ptr(stream)))
    return float(fl.value)


def probe_mfma_varied(ctx: Context, iters: int, out: torch.Tensor, stream=None) -> float:
    """BF16 MFMA-only loop on lane- and element-varying operands (libmrf
    mrf_probe_mfma_varied). Returns the flops the launch performs; it does
    not wait."""
    if out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 CUDA tensor")
    fl = C.c_double()
    L.check(ctx._lib.mrf_probe_mfma_varied(ctx.handle, int(iters), out.data_ptr(), out.numel(),
                                           C.byref(fl), _stream_ptr(stream)))
    return float(fl.value)


def probe_write(ctx: Context, dst: torch.Tensor, pattern: int = 0x5A5A5A5A, stream=None) -> int:
    """Fill a contiguous CUDA tensor with non-temporal 16 B stores (libmrf
    mrf_probe_write). Returns the bytes written; it does not wait."""
    if not dst.is_cuda or not dst.is_contiguous():
        raise ValueError("dst must be a contiguous CUDA tensor")
    nbytes = dst.numel() * dst.element_size()
    L.check(ctx._lib.mrf_probe_write(ctx.handle, dst.data_ptr(), nbytes, int(pattern) & 0xFFFFFFFF,
                                     _stream_ptr(stream)))
    return nbytes
