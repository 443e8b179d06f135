"""ctypes binding of libkbisim.so (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libkbisim.so")

KBISIM_MEM_HOST = 0
KBISIM_MEM_DEVICE = 1
PROF_CLASSES = ["signature", "order", "assign", "round"]
WORK_BUCKETS = ["thread", "wave", "block", "hub"]

REQUEST_STATES = ["queued", "running", "done", "failed", "cancelled"]
STATUS = {0: "KBISIM_OK", -1: "KBISIM_EINVAL", -2: "KBISIM_ENOMEM", -3: "KBISIM_EDEVICE",
          -4: "KBISIM_ESTATE", -5: "KBISIM_EBUSY", -6: "KBISIM_ECANCELED", -7: "KBISIM_ETIMEDOUT"}


class KbisimError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


class GraphDesc(ctypes.Structure):
    _fields_ = [("num_nodes", ctypes.c_int64), ("num_edges", ctypes.c_int64),
                ("node_label", ctypes.c_void_p), ("edge_src", ctypes.c_void_p),
                ("edge_label", ctypes.c_void_p), ("edge_dst", ctypes.c_void_p),
                ("mem", ctypes.c_int), ("stream", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("early_stop", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("medium_cap", ctypes.c_int32), ("history", ctypes.c_int32),
                ("update_mode", ctypes.c_int32), ("radix_tile", ctypes.c_int32),
                ("edge_window_bytes", ctypes.c_int64)]


class UpdateDesc(ctypes.Structure):
    _fields_ = [("num_new_nodes", ctypes.c_int64), ("new_node_label", ctypes.c_void_p),
                ("num_del_edges", ctypes.c_int64), ("del_src", ctypes.c_void_p),
                ("del_label", ctypes.c_void_p), ("del_dst", ctypes.c_void_p),
                ("num_del_nodes", ctypes.c_int64), ("del_nodes", ctypes.c_void_p),
                ("num_add_edges", ctypes.c_int64), ("add_src", ctypes.c_void_p),
                ("add_label", ctypes.c_void_p), ("add_dst", ctypes.c_void_p),
                ("mem", ctypes.c_int)]


_lib = None


def lib_path():
    return _LIB_PATH


def load_library():
    """Loads libkbisim.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError("libkbisim.so not built: run `python -m paper_1210_0748_amd.build` "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.kbisim_options_default.argtypes = [ctypes.POINTER(Options)]
    lib.kbisim_options_default.restype = None
    lib.kbisim_create.argtypes = [ctypes.POINTER(GraphDesc), ctypes.POINTER(Options), ctypes.POINTER(vp)]
    lib.kbisim_create.restype = ctypes.c_int
    lib.kbisim_refine.argtypes = [vp, i32, ctypes.POINTER(i32)]
    lib.kbisim_refine.restype = ctypes.c_int
    lib.kbisim_result.argtypes = [vp, vp, ctypes.c_int, ctypes.POINTER(i64), vp, i32]
    lib.kbisim_result.restype = ctypes.c_int
    lib.kbisim_refine_static.argtypes = [ctypes.POINTER(GraphDesc), i32, ctypes.POINTER(Options), vp, ctypes.c_int,
                                         ctypes.POINTER(i64), ctypes.POINTER(i32)]
    lib.kbisim_refine_static.restype = ctypes.c_int
    lib.kbisim_stream_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32)]
    lib.kbisim_stream_stats.restype = ctypes.c_int
    lib.kbisim_result_round.argtypes = [vp, i32, vp, ctypes.c_int, ctypes.POINTER(i64)]
    lib.kbisim_result_round.restype = ctypes.c_int
    lib.kbisim_update.argtypes = [vp, ctypes.POINTER(UpdateDesc), ctypes.POINTER(i32)]
    lib.kbisim_update.restype = ctypes.c_int
    lib.kbisim_update_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                        ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.kbisim_update_stats.restype = ctypes.c_int
    lib.kbisim_profile.argtypes = [vp, vp, vp, i32, i32]
    lib.kbisim_profile.restype = ctypes.c_int
    lib.kbisim_work.argtypes = [vp, vp, i32, i32]
    lib.kbisim_work.restype = ctypes.c_int
    lib.kbisim_round_profile.argtypes = [vp, ctypes.POINTER(RoundStat), i32, ctypes.POINTER(i32), i32]
    lib.kbisim_round_profile.restype = ctypes.c_int
    lib.kbisim_release_cached.argtypes = [ctypes.POINTER(i64)]
    lib.kbisim_release_cached.restype = ctypes.c_int
    lib.kbisim_batch_create.argtypes = [i32, vp, vp, ctypes.POINTER(GraphDesc), ctypes.POINTER(Options),
                                        ctypes.POINTER(vp)]
    lib.kbisim_batch_create.restype = ctypes.c_int
    lib.kbisim_batch_refine.argtypes = [vp, vp, vp]
    lib.kbisim_batch_refine.restype = ctypes.c_int
    lib.kbisim_batch_result.argtypes = [vp, vp, ctypes.c_int, vp]
    lib.kbisim_batch_result.restype = ctypes.c_int
    lib.kbisim_batch_destroy.argtypes = [vp]
    lib.kbisim_batch_destroy.restype = None
    u64 = ctypes.c_uint64
    lib.kbisim_server_create.argtypes = [u64, i32, ctypes.POINTER(Options), ctypes.POINTER(vp)]
    lib.kbisim_server_create.restype = ctypes.c_int
    lib.kbisim_server_submit.argtypes = [vp, ctypes.POINTER(GraphDesc), i32, ctypes.POINTER(u64)]
    lib.kbisim_server_submit.restype = ctypes.c_int
    lib.kbisim_server_wait.argtypes = [vp, u64, vp, ctypes.c_int, ctypes.POINTER(i64), ctypes.POINTER(i32),
                                       ctypes.c_double]
    lib.kbisim_server_wait.restype = ctypes.c_int
    lib.kbisim_server_cancel.argtypes = [vp, u64]
    lib.kbisim_server_cancel.restype = ctypes.c_int
    lib.kbisim_server_timing.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.kbisim_server_timing.restype = ctypes.c_int
    lib.kbisim_server_release.argtypes = [vp, u64]
    lib.kbisim_server_release.restype = ctypes.c_int
    lib.kbisim_server_state.argtypes = [vp, u64, ctypes.POINTER(i32)]
    lib.kbisim_server_state.restype = ctypes.c_int
    lib.kbisim_server_in_use.argtypes = [vp, ctypes.POINTER(u64)]
    lib.kbisim_server_in_use.restype = ctypes.c_int
    lib.kbisim_server_destroy.argtypes = [vp]
    lib.kbisim_server_destroy.restype = None
    lib.kbisim_destroy.argtypes = [vp]
    lib.kbisim_destroy.restype = None
    lib.kbisim_status_str.argtypes = [ctypes.c_int]
    lib.kbisim_status_str.restype = ctypes.c_char_p
    lib.kbisim_last_error.argtypes = []
    lib.kbisim_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(st):
    if st != 0:
        lib = load_library()
        raise KbisimError(st, lib.kbisim_last_error().decode())


def kbisim_status_str(status):
    return load_library().kbisim_status_str(int(status)).decode()


def kbisim_last_error():
    return load_library().kbisim_last_error().decode()


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _arrays(node_label, src, elab, dst):
    """Returns (mem kind, pointers, keepalive) for torch CUDA tensors or numpy."""
    try:
        import torch
        is_torch = isinstance(node_label, torch.Tensor)
    except ImportError:  # pragma: no cover
        is_torch = False
    if is_torch:
        arrs = []
        dev = None
        for a in (node_label, src, elab, dst):
            if a.dtype != torch.int32:
                raise TypeError("arrays must be int32")
            if not a.is_cuda:
                raise TypeError("torch tensors must be on the GPU (use numpy for host arrays)")
            if dev is not None and a.device != dev:
                raise TypeError("all arrays must be on one device")
            dev = a.device
            arrs.append(a.contiguous())
        return KBISIM_MEM_DEVICE, [a.data_ptr() for a in arrs], arrs
    arrs = [np.ascontiguousarray(np.asarray(a), dtype=np.int32) for a in (node_label, src, elab, dst)]
    return KBISIM_MEM_HOST, [a.ctypes.data for a in arrs], arrs


def kbisim_create(num_nodes, node_label, src, elab, dst, *, stream=None, early_stop=True,
                  profile=False, medium_cap=None, history=False, update_mode=0, edge_window_bytes=0,
                  radix_tile=0):
    """Creates a device-resident graph handle (see kbisim.h). Returns the handle.
    edge_window_bytes > 0 keeps the edge table (host arrays) in host memory and
    streams it through device windows of that total size every round."""
    lib = load_library()
    mem, ptrs, keep = _arrays(node_label, src, elab, dst)
    n, m = int(num_nodes), int(keep[1].shape[0])
    if int(keep[0].shape[0]) != n or int(keep[2].shape[0]) != m or int(keep[3].shape[0]) != m:
        raise KbisimError(-1, "array lengths do not match num_nodes / num_edges")
    desc = GraphDesc(n, m, ptrs[0] or None, ptrs[1] or None, ptrs[2] or None, ptrs[3] or None, mem,
                     _stream_ptr(stream))
    opt = Options()
    lib.kbisim_options_default(ctypes.byref(opt))
    opt.early_stop = 1 if early_stop else 0
    opt.profile = 1 if profile else 0
    opt.history = 1 if history else 0
    opt.update_mode = int(update_mode)
    opt.edge_window_bytes = int(edge_window_bytes)
    opt.radix_tile = int(radix_tile)
    if medium_cap is not None:
        opt.medium_cap = int(medium_cap)
    h = ctypes.c_void_p()
    _check(lib.kbisim_create(ctypes.byref(desc), ctypes.byref(opt), ctypes.byref(h)))
    return h


def kbisim_stream_stats(handle):
    """(partitions, bytes of the edge table moved host->device by the rounds,
    rounds that read their active rows in place) of a streamed graph."""
    p, b, d = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int32(0)
    _check(load_library().kbisim_stream_stats(handle, ctypes.byref(p), ctypes.byref(b), ctypes.byref(d)))
    return int(p.value), int(b.value), int(d.value)


def kbisim_refine(handle, k):
    rd = ctypes.c_int32(0)
    _check(load_library().kbisim_refine(handle, int(k), ctypes.byref(rd)))
    return int(rd.value)


def kbisim_result(handle, pid_out=None, counts_cap=0):
    """pid_out: torch CUDA int32 tensor, numpy int32 array or None.
    Returns (num_blocks, counts list)."""
    lib = load_library()
    nb = ctypes.c_int64(0)
    counts = np.zeros(max(int(counts_cap), 0), np.int64)
    mem, ptr = KBISIM_MEM_HOST, None
    if pid_out is not None:
        if isinstance(pid_out, np.ndarray):
            assert pid_out.dtype == np.int32 and pid_out.flags.c_contiguous
            ptr = pid_out.ctypes.data
        else:
            assert pid_out.dtype.__repr__().endswith("int32") and pid_out.is_contiguous()
            mem, ptr = KBISIM_MEM_DEVICE, pid_out.data_ptr()
    _check(lib.kbisim_result(handle, ptr, mem, ctypes.byref(nb),
                             counts.ctypes.data if counts_cap else None, int(counts_cap)))
    return int(nb.value), [int(c) for c in counts]


def _out_ptr(pid_out):
    if pid_out is None:
        return KBISIM_MEM_HOST, None
    if isinstance(pid_out, np.ndarray):
        assert pid_out.dtype == np.int32 and pid_out.flags.c_contiguous
        return KBISIM_MEM_HOST, (pid_out.ctypes.data if pid_out.size else None)
    assert pid_out.dtype.__repr__().endswith("int32") and pid_out.is_contiguous()
    return KBISIM_MEM_DEVICE, (pid_out.data_ptr() if pid_out.numel() else None)


def kbisim_result_round(handle, round_, pid_out=None):
    """Ids of round `round_` (change of k) into pid_out; returns B of that round."""
    mem, ptr = _out_ptr(pid_out)
    nb = ctypes.c_int64(0)
    _check(load_library().kbisim_result_round(handle, int(round_), ptr, mem, ctypes.byref(nb)))
    return int(nb.value)


def kbisim_update(handle, *, new_labels=None, delete=None, delete_nodes=None, add=None):
    """Applies one update (see kbisim.h): new_labels (new nodes), delete and
    add as (src, label, dst) triples of arrays, delete_nodes (node ids);
    numpy (host) or torch CUDA int32 tensors (device), all of one kind.
    Returns rounds done."""
    parts = []
    for a in ([new_labels] if new_labels is not None else []) + list(delete or ()) + list(add or ()) + \
            ([delete_nodes] if delete_nodes is not None else []):
        parts.append(a)
    is_dev = False
    try:
        import torch
        is_dev = any(isinstance(a, torch.Tensor) for a in parts)
    except ImportError:  # pragma: no cover
        pass
    keep = []

    def arr(a):
        if a is None:
            return 0, None
        if is_dev:
            if str(a.dtype) != "torch.int32" or not a.is_cuda:
                raise TypeError("device update arrays must be int32 CUDA tensors")
            t = a.contiguous()
            keep.append(t)
            return int(t.numel()), (t.data_ptr() if t.numel() else None)
        x = np.ascontiguousarray(np.asarray(a), dtype=np.int32)
        keep.append(x)
        return int(x.shape[0]), (x.ctypes.data if x.size else None)

    n_new, p_new = arr(new_labels)
    d = [arr(x) for x in (delete if delete is not None else (None, None, None))]
    a = [arr(x) for x in (add if add is not None else (None, None, None))]
    n_dn, p_dn = arr(delete_nodes)
    if len({x[0] for x in d}) > 1 or len({x[0] for x in a}) > 1:
        raise KbisimError(-1, "edge arrays of different lengths")
    desc = UpdateDesc(n_new, p_new, d[0][0], d[0][1], d[1][1], d[2][1], n_dn, p_dn, a[0][0], a[0][1], a[1][1],
                      a[2][1], KBISIM_MEM_DEVICE if is_dev else KBISIM_MEM_HOST)
    rd = ctypes.c_int32(0)
    _check(load_library().kbisim_update(handle, ctypes.byref(desc), ctypes.byref(rd)))
    return int(rd.value)


def kbisim_refine_static(num_nodes, node_label, src, elab, dst, k, pid_out, *, stream=None, early_stop=True,
                         medium_cap=None, radix_tile=0):
    """The allocation-free one-shot refine (static scratch region): ids of
    round k (or the fixed point) into pid_out (numpy or torch CUDA int32).
    Returns (num_blocks, rounds_done)."""
    lib = load_library()
    mem, ptrs, keep = _arrays(node_label, src, elab, dst)
    n, m = int(num_nodes), int(keep[1].shape[0])
    desc = GraphDesc(n, m, ptrs[0] or None, ptrs[1] or None, ptrs[2] or None, ptrs[3] or None, mem,
                     _stream_ptr(stream) if (mem == KBISIM_MEM_DEVICE or stream is not None) else None)
    opt = _options(early_stop=early_stop, medium_cap=medium_cap, radix_tile=radix_tile)
    out_mem, out_ptr = _out_ptr(pid_out)
    nb, rd = ctypes.c_int64(0), ctypes.c_int32(0)
    _check(lib.kbisim_refine_static(ctypes.byref(desc), int(k), ctypes.byref(opt), out_ptr, out_mem,
                                    ctypes.byref(nb), ctypes.byref(rd)))
    return int(nb.value), int(rd.value)


def kbisim_update_stats(handle):
    """(levels, full_from, rechecked, recomputed, changed) of the last update."""
    v = [ctypes.c_int64(0) for _ in range(5)]
    _check(load_library().kbisim_update_stats(handle, *[ctypes.byref(x) for x in v]))
    return tuple(int(x.value) for x in v)


def kbisim_profile(handle, reset=False):
    n = len(PROF_CLASSES)
    ms = np.zeros(n, np.float64)
    cnt = np.zeros(n, np.int64)
    _check(load_library().kbisim_profile(handle, ms.ctypes.data, cnt.ctypes.data, n, 1 if reset else 0))
    return {c: (float(ms[i]), int(cnt[i])) for i, c in enumerate(PROF_CLASSES)}


def kbisim_work(handle, reset=False):
    """Per signature bucket: (active nodes, their edges), summed over rounds."""
    w = np.zeros(8, np.int64)
    _check(load_library().kbisim_work(handle, w.ctypes.data, 8, 1 if reset else 0))
    return {WORK_BUCKETS[c]: (int(w[2 * c]), int(w[2 * c + 1])) for c in range(4)}


class RoundStat(ctypes.Structure):
    _fields_ = [("signature_ms", ctypes.c_double), ("round_ms", ctypes.c_double),
                ("active_nodes", ctypes.c_int64), ("active_edges", ctypes.c_int64),
                ("max_keys", ctypes.c_int64)]


def kbisim_round_profile(handle, reset=False, cap=64):
    """Per round (profile mode): dicts with signature_ms, round_ms,
    active_nodes, active_edges, max_keys."""
    buf = (RoundStat * cap)()
    n = ctypes.c_int32(0)
    _check(load_library().kbisim_round_profile(handle, buf, cap, ctypes.byref(n), 1 if reset else 0))
    return [{f: getattr(buf[r], f) for f, _ in RoundStat._fields_} for r in range(min(n.value, cap))]


def kbisim_release_cached():
    """Frees the library's cache of device memory; returns the bytes released."""
    b = ctypes.c_int64(0)
    _check(load_library().kbisim_release_cached(ctypes.byref(b)))
    return int(b.value)


def kbisim_destroy(handle):
    if handle:
        load_library().kbisim_destroy(handle)


class Graph:
    """Owning wrapper of a kbisim handle."""

    def __init__(self, num_nodes, node_label, src, elab, dst, **kw):
        self.num_nodes = int(num_nodes)
        self._h = kbisim_create(num_nodes, node_label, src, elab, dst, **kw)
        self.rounds_done = 0

    def refine(self, k):
        self.rounds_done = kbisim_refine(self._h, k)
        return self.rounds_done

    def result(self, device=None):
        """Ids of the last round: a torch CUDA tensor if `device` is given,
        else a numpy array. Also returns (num_blocks, counts)."""
        cap = self.rounds_done + 1
        if device is not None:
            import torch
            out = torch.empty(self.num_nodes, dtype=torch.int32, device=device)
        else:
            out = np.empty(self.num_nodes, np.int32)
        nb, counts = kbisim_result(self._h, out if self.num_nodes else None, cap)
        return out, nb, counts

    def result_round(self, round_, device=None):
        """Ids of an earlier round (history option) or the current one:
        (ids, num_blocks)."""
        if device is not None:
            import torch
            out = torch.empty(self.num_nodes, dtype=torch.int32, device=device)
        else:
            out = np.empty(self.num_nodes, np.int32)
        nb = kbisim_result_round(self._h, round_, out)
        return out, nb

    def update(self, *, new_labels=None, delete=None, delete_nodes=None, add=None):
        """Applies an update (history option); returns rounds done."""
        self.rounds_done = kbisim_update(self._h, new_labels=new_labels, delete=delete, delete_nodes=delete_nodes,
                                         add=add)
        if new_labels is not None:
            self.num_nodes += int(len(new_labels))
        if delete_nodes is not None and len(delete_nodes):
            self.num_nodes -= int(np.unique(np.asarray(
                delete_nodes.cpu() if hasattr(delete_nodes, "cpu") else delete_nodes)).size)
        return self.rounds_done

    def update_stats(self):
        return kbisim_update_stats(self._h)

    def profile(self, reset=False):
        return kbisim_profile(self._h, reset)

    def work(self, reset=False):
        return kbisim_work(self._h, reset)

    def round_profile(self, reset=False):
        return kbisim_round_profile(self._h, reset)

    def close(self):
        if self._h:
            kbisim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def refine(num_nodes, node_label, src, elab, dst, k, **kw):
    """One-shot: returns (pid numpy array, counts, rounds_done)."""
    with Graph(num_nodes, node_label, src, elab, dst, **kw) as g:
        rd = g.refine(k)
        pid, _, counts = g.result()
        return pid, counts, rd


def _options(early_stop=True, profile=False, medium_cap=None, history=False, radix_tile=0):
    lib = load_library()
    opt = Options()
    lib.kbisim_options_default(ctypes.byref(opt))
    opt.early_stop = 1 if early_stop else 0
    opt.profile = 1 if profile else 0
    opt.history = 1 if history else 0
    opt.radix_tile = int(radix_tile)
    if medium_cap is not None:
        opt.medium_cap = int(medium_cap)
    return opt


def kbisim_batch_create(node_off, edge_off, node_label, src, elab, dst, *, stream=None, **kw):
    """Batch of graphs concatenated in the four arrays (local endpoint ids);
    node_off / edge_off: num_graphs + 1 offsets. Returns the handle."""
    lib = load_library()
    mem, ptrs, keep = _arrays(node_label, src, elab, dst)
    noff = np.ascontiguousarray(np.asarray(node_off, dtype=np.int64))
    eoff = np.ascontiguousarray(np.asarray(edge_off, dtype=np.int64))
    G = int(noff.shape[0]) - 1
    desc = GraphDesc(int(noff[-1]), int(eoff[-1]), ptrs[0] or None, ptrs[1] or None, ptrs[2] or None,
                     ptrs[3] or None, mem, _stream_ptr(stream))
    opt = _options(**kw)
    h = ctypes.c_void_p()
    _check(lib.kbisim_batch_create(G, noff.ctypes.data, eoff.ctypes.data, ctypes.byref(desc),
                                   ctypes.byref(opt), ctypes.byref(h)))
    return h, G


def kbisim_batch_refine(handle, k_per_graph):
    k = np.ascontiguousarray(np.asarray(k_per_graph, dtype=np.int32))
    rd = np.zeros(k.shape[0], np.int32)
    _check(load_library().kbisim_batch_refine(handle, k.ctypes.data, rd.ctypes.data))
    return rd


def kbisim_batch_result(handle, num_graphs, pid_out):
    """pid_out: numpy int32 array or torch CUDA int32 tensor of sum N. Returns blocks per graph."""
    blocks = np.zeros(num_graphs, np.int64)
    if isinstance(pid_out, np.ndarray):
        mem, ptr = KBISIM_MEM_HOST, (pid_out.ctypes.data if pid_out.size else None)
    else:
        mem, ptr = KBISIM_MEM_DEVICE, (pid_out.data_ptr() if pid_out.numel() else None)
    _check(load_library().kbisim_batch_result(handle, ptr, mem, blocks.ctypes.data))
    return blocks


def kbisim_batch_destroy(handle):
    if handle:
        load_library().kbisim_batch_destroy(handle)


def refine_batch(graphs, k, device=None, **kw):
    """Refines a list of graphs (objects with num_nodes, node_label, src, elab,
    dst) as one batch. k: int or per-graph list. Returns (list of id arrays,
    blocks, rounds_done)."""
    noff = np.zeros(len(graphs) + 1, np.int64)
    eoff = np.zeros(len(graphs) + 1, np.int64)
    for i, g in enumerate(graphs):
        noff[i + 1] = noff[i] + int(g.num_nodes)
        eoff[i + 1] = eoff[i] + int(np.asarray(g.src).shape[0])
    cat = lambda name: np.concatenate([np.asarray(getattr(g, name), np.int32) for g in graphs]) \
        if graphs else np.zeros(0, np.int32)
    arrs = [cat("node_label"), cat("src"), cat("elab"), cat("dst")]
    if device is not None:
        import torch
        arrs = [torch.from_numpy(a).to(device) for a in arrs]
    ks = [int(k)] * len(graphs) if np.isscalar(k) else list(k)
    h, G = kbisim_batch_create(noff, eoff, *arrs, **kw)
    try:
        rd = kbisim_batch_refine(h, ks)
        out = np.empty(int(noff[-1]), np.int32)
        blocks = kbisim_batch_result(h, G, out)
    finally:
        kbisim_batch_destroy(h)
    pids = [out[noff[i]:noff[i + 1]] for i in range(len(graphs))]
    return pids, [int(b) for b in blocks], [int(r) for r in rd]


class Server:
    """Binding of the served form (kbisim_server_*)."""

    def __init__(self, hbm_budget_bytes, max_slots=4, **kw):
        lib = load_library()
        opt = _options(**kw)
        h = ctypes.c_void_p()
        _check(lib.kbisim_server_create(int(hbm_budget_bytes), int(max_slots), ctypes.byref(opt),
                                        ctypes.byref(h)))
        self._h = h
        self._keep = {}
        self._n = {}

    def submit(self, num_nodes, node_label, src, elab, dst, k):
        """Host arrays are copied; device (torch) arrays are referenced and
        kept alive here until the request has been waited for."""
        mem, ptrs, keep = _arrays(node_label, src, elab, dst)
        n, m = int(num_nodes), int(keep[1].shape[0])
        stream = _stream_ptr(None) if mem == KBISIM_MEM_DEVICE else None
        desc = GraphDesc(n, m, ptrs[0] or None, ptrs[1] or None, ptrs[2] or None, ptrs[3] or None, mem, stream)
        rid = ctypes.c_uint64(0)
        _check(load_library().kbisim_server_submit(self._h, ctypes.byref(desc), int(k), ctypes.byref(rid)))
        if mem == KBISIM_MEM_DEVICE:
            self._keep[rid.value] = keep
        self._n[rid.value] = n
        return int(rid.value)

    def wait(self, rid, timeout_s=-1.0):
        """Returns (ids numpy array, num_blocks, rounds_done); raises KbisimError."""
        n = self._n[rid]
        out = np.empty(n, np.int32)
        nb = ctypes.c_int64(0)
        rd = ctypes.c_int32(0)
        st = load_library().kbisim_server_wait(self._h, int(rid), out.ctypes.data if n else None,
                                               KBISIM_MEM_HOST, ctypes.byref(nb), ctypes.byref(rd),
                                               float(timeout_s))
        if st != -7:  # anything but a time-out ends the request's use of its inputs
            self._keep.pop(rid, None)
        _check(st)
        return out, int(nb.value), int(rd.value)

    def cancel(self, rid):
        _check(load_library().kbisim_server_cancel(self._h, int(rid)))

    def timing(self, rid):
        q, t = ctypes.c_double(0), ctypes.c_double(0)
        _check(load_library().kbisim_server_timing(self._h, int(rid), ctypes.byref(q), ctypes.byref(t)))
        return q.value, t.value

    def release(self, rid):
        _check(load_library().kbisim_server_release(self._h, int(rid)))
        self._n.pop(rid, None)

    def state(self, rid):
        """One of REQUEST_STATES (queued, running, done, failed, cancelled)."""
        st = ctypes.c_int32(0)
        _check(load_library().kbisim_server_state(self._h, int(rid), ctypes.byref(st)))
        return REQUEST_STATES[st.value]

    def in_use(self):
        b = ctypes.c_uint64(0)
        _check(load_library().kbisim_server_in_use(self._h, ctypes.byref(b)))
        return int(b.value)

    def close(self):
        if self._h:
            load_library().kbisim_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
