"""Python binding of libnd (MI355X network density of states).

Argument marshalling only: every computation runs in the HIP library through
its C ABI (``include/nd.h``); PyTorch supplies device memory and streams.  The
functions carry the C names.  Device outputs are caller-allocated torch
tensors (checked here for device, dtype, contiguity and size before any
pointer crosses the ABI); host outputs come back as numpy arrays.

Importing the package loads ``libnd.so`` (built in-tree by
``python -m paper_1905_09758_amd.build``); if it is missing the import fails
loudly -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnd.so")

ND_OK, ND_EINVAL, ND_ENOMEM, ND_EDEVICE, ND_EOVERFLOW, ND_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
ND_INPUT_DEVICE = 0x1
ND_PROBE_RADEMACHER, ND_PROBE_GAUSSIAN, ND_STATE_FP64, ND_TIME_STEPS = 0x0, 0x1, 0x2, 0x4
ND_MOMENT_DOUBLING = 0x8
ND_TWINS_OPEN = 0x1
ND_TWINS_CLOSED = 0x2
ND_PENDANTS = 0x4
ND_HUBPATHS = 0x8
ND_KERNEL_NONE, ND_KERNEL_JACKSON, ND_SPIKES_IN_MOMENTS = 0, 1, 0x10

_STATUS = {ND_EINVAL: "ND_EINVAL", ND_ENOMEM: "ND_ENOMEM", ND_EDEVICE: "ND_EDEVICE",
           ND_EOVERFLOW: "ND_EOVERFLOW", ND_EUNSUPPORTED: "ND_EUNSUPPORTED"}

# every symbol the C header declares (checked by the CPU test suite)
EXPORTS = (
    "nd_build_csr", "nd_graph_info", "nd_graph_export", "nd_graph_device_arrays", "nd_graph_step_timing",
    "nd_graph_free",
    "nd_motif_filter", "nd_motif_info", "nd_motif_export", "nd_motif_export_lambda", "nd_motifs_free",
    "nd_make_probes",
    "nd_cheb_moments", "nd_cheb_moments_noalloc", "nd_ldos_moments", "nd_pdos_nodes", "nd_pdos_nested", "nd_nested_tree", "nd_gql", "nd_gql_pdos", "nd_gql_density", "nd_reconstruct", "nd_node_features", "nd_cv_exact_diag", "nd_motif_diag", "nd_ldos_variance", "nd_column_stats",
    "nd_mlp_forward", "nd_mlp_grad", "nd_adam_step", "nd_last_error",
)


class NDError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__("%s: %s (%s)" % (where, _STATUS.get(status, str(status)), msg))
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError("libnd.so is not built (%s); run `python paper_1905_09758_amd/build.py`" % LIB_PATH)

# torch first: libnd then binds to the HIP runtime torch has already loaded
# (same soname), so device memory and streams are shared with torch's.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)
_vp, _i64, _i32, _u32, _u64, _dbl, _flt = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                                           ctypes.c_uint64, ctypes.c_double, ctypes.c_float)
_P = ctypes.POINTER


def _sig(name, args, res=ctypes.c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_sig("nd_build_csr", [_i64, _i64, _vp, _vp, _u32, _vp, _P(_vp)])
_sig("nd_graph_info", [_vp, _P(_i64), _P(_i64), _P(_i64)])
_sig("nd_graph_export", [_vp, _vp, _vp, _vp, _vp])
_sig("nd_graph_device_arrays", [_vp, _P(_vp), _P(_vp), _P(_vp)])
_sig("nd_graph_step_timing", [_vp, _P(_dbl), _P(_i64)])
_sig("nd_graph_free", [_vp], None)
_sig("nd_motif_filter", [_vp, _u64, _u32, _vp, _P(_vp)])
_sig("nd_motif_info", [_vp, _P(_i64), _P(_i64), _P(_i32), _vp, _vp])
_sig("nd_motif_export", [_vp, _vp, _vp])
_sig("nd_motif_export_lambda", [_vp, _vp, _vp])
_sig("nd_motifs_free", [_vp], None)
_sig("nd_make_probes", [_vp, _vp, _i32, _u64, _u32, _vp, _vp])
_sig("nd_cheb_moments", [_vp, _vp, _i32, _i32, _u64, _u32, _vp, _vp, _vp])
_sig("nd_cheb_moments_noalloc", [_vp, _i32, _i32, _u64, _u32, _vp, _vp, _vp])
_sig("nd_ldos_moments", [_vp, _vp, _i32, _i32, _u64, _u32, _vp, _vp, _vp, _vp, _vp])
_sig("nd_pdos_nodes", [_vp, _vp, _i32, _i32, _u32, _vp, _vp])
_sig("nd_pdos_nested", [_vp, _i32, _i32, _i64, _u32, _vp, _vp, _vp])
_sig("nd_nested_tree", [_vp, _vp, _i64, _i32, _vp, _vp, _vp])
_sig("nd_gql", [_vp, _vp, _i32, _i32, _u64, _u32, _vp, _vp, _vp, _vp, _vp, _vp])
_sig("nd_gql_pdos", [_vp, _vp, _i32, _i32, _u32, _vp, _vp, _vp, _vp])
_sig("nd_gql_density", [_vp, _vp, _i32, _i32, _i32, _vp, _i32, _dbl, _dbl, _vp, _vp])
_sig("nd_reconstruct", [_vp, _i64, _i32, _u32, _vp, _vp, _i32, _i32, _dbl, _dbl, _vp, _i32, _vp, _vp])
_sig("nd_last_error", [], ctypes.c_char_p)
_sig("nd_node_features", [_vp, _vp, _vp, _vp, _vp])
_sig("nd_cv_exact_diag", [_vp, _vp, _i64, _i32, _vp])
_sig("nd_motif_diag", [_vp, _vp, _i64, _i32, ctypes.c_double, _vp])
_sig("nd_ldos_variance", [_vp, _vp, _i64, _i32, _i32, _i32, _vp, _vp, _vp])
_sig("nd_column_stats", [_vp, _i64, _i32, _vp, _vp, _vp])
_sig("nd_mlp_forward", [_vp, _vp, _i64, _i32, _vp, _vp])
_sig("nd_mlp_grad", [_vp, _vp, _vp, _i32, _vp, _i64, _i32, _vp, _vp, _vp])
_sig("nd_adam_step", [_vp, _vp, _vp, _vp, _i64, _i32, _flt, _vp])


def _check(status: int, where: str):
    if status != ND_OK:
        raise NDError(status, where, _lib.nd_last_error().decode())


def lib():
    return _lib


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible")


# ------------------------------------------------------------------ helpers
def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, numel, name):
    """Pointer of a contiguous device tensor with at least `numel` elements."""
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < numel:
        raise ValueError("%s holds %d elements, needs %d" % (name, t.numel(), numel))
    return ctypes.c_void_p(t.data_ptr())


class Graph:
    """Owns an nd_graph handle."""

    def __init__(self, handle):
        self.handle = handle
        n, nnz, mx = _i64(), _i64(), _i64()
        _check(_lib.nd_graph_info(handle, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(mx)), "nd_graph_info")
        self.n, self.nnz, self.max_deg = n.value, nnz.value, mx.value

    def __del__(self, _free=_lib.nd_graph_free):
        h = getattr(self, "handle", None)
        if h:
            _free(h)
            self.handle = None


class Motifs:
    """Owns an nd_motifs handle."""

    def __init__(self, handle, graph):
        self.handle = handle
        self.graph = graph
        info = nd_motif_info(self)
        self.n_classes, self.n_members = info["n_classes"], info["n_members"]
        self.spikes = info["spikes"]

    def __del__(self, _free=_lib.nd_motifs_free):
        h = getattr(self, "handle", None)
        if h:
            _free(h)
            self.handle = None


def _h(x):
    return None if x is None else x.handle


# ------------------------------------------------------------------ graph
def nd_build_csr(n_nodes: int, src, dst, stream=None) -> Graph:
    """src/dst: int32 numpy arrays (host) or int32 device tensors."""
    import torch
    flags = 0
    if isinstance(src, torch.Tensor):
        if src.is_cuda != dst.is_cuda:
            raise ValueError("src and dst must live on the same side")
        if src.is_cuda:
            flags |= ND_INPUT_DEVICE
            m = src.numel()
            ps, pd = _dev(src, torch.int32, m, "src"), _dev(dst, torch.int32, m, "dst")
            keep = (src, dst)
        else:
            src, dst = src.numpy(), dst.numpy()
    if not flags:
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        m = src.size
        if dst.size != m:
            raise ValueError("src/dst length mismatch")
        ps, pd = ctypes.c_void_p(src.ctypes.data), ctypes.c_void_p(dst.ctypes.data)
        keep = (src, dst)
    if flags and dst.numel() != m:
        raise ValueError("src/dst length mismatch")
    out = _vp()
    _check(_lib.nd_build_csr(n_nodes, m, ps, pd, flags, _stream(stream), ctypes.byref(out)), "nd_build_csr")
    del keep
    return Graph(out)


def nd_graph_info(g: Graph):
    return g.n, g.nnz, g.max_deg


def nd_graph_step_timing(g: Graph):
    """(total ms, launches) of the step kernels of the last call made with ND_TIME_STEPS."""
    ms, n = _dbl(), _i64()
    _check(_lib.nd_graph_step_timing(g.handle, ctypes.byref(ms), ctypes.byref(n)), "nd_graph_step_timing")
    return ms.value, n.value


def nd_graph_export(g: Graph) -> dict:
    rp = np.empty(g.n + 1, np.int64)
    col = np.empty(max(g.nnz, 1), np.int32)
    old = np.empty(max(g.n, 1), np.int32)
    dinv = np.empty(max(g.n, 1), np.float32)
    _check(_lib.nd_graph_export(g.handle, rp.ctypes.data, col.ctypes.data, old.ctypes.data, dinv.ctypes.data),
           "nd_graph_export")
    return {"row_ptr": rp, "col": col[:g.nnz], "old_id": old[:g.n], "dinv_sqrt": dinv[:g.n]}


# ------------------------------------------------------------------ motifs
def nd_motif_filter(g: Graph, seed: int, kinds: int = ND_TWINS_OPEN, stream=None) -> Motifs:
    out = _vp()
    _check(_lib.nd_motif_filter(g.handle, seed, kinds, _stream(stream), ctypes.byref(out)), "nd_motif_filter")
    return Motifs(out, g)


def nd_motif_info(m: Motifs) -> dict:
    nc, nm, ns = _i64(), _i64(), _i32()
    _check(_lib.nd_motif_info(m.handle, ctypes.byref(nc), ctypes.byref(nm), ctypes.byref(ns), None, None),
           "nd_motif_info")
    lam = np.empty(max(ns.value, 1), np.float64)
    w = np.empty(max(ns.value, 1), np.float64)
    _check(_lib.nd_motif_info(m.handle, None, None, None, lam.ctypes.data, w.ctypes.data), "nd_motif_info")
    spikes = [(float(lam[i]), float(w[i])) for i in range(ns.value)]
    return {"n_classes": nc.value, "n_members": nm.value, "spikes": spikes}


def nd_motif_export(m: Motifs):
    ptr = np.empty(m.n_classes + 1, np.int64)
    mem = np.empty(max(m.n_members, 1), np.int32)
    _check(_lib.nd_motif_export(m.handle, ptr.ctypes.data, mem.ctypes.data), "nd_motif_export")
    return ptr, mem[:m.n_members]


def nd_motif_export_lambda(m: Motifs, paired: bool = False):
    """Eigenvalue removed by each class: 0 (open twins), -1/d (closed twins)
    or 1/sqrt(d) (pendant-twin classes); with paired=True also the int32
    flags of the classes that hold +-lambda."""
    lam = np.empty(max(m.n_classes, 1), np.float64)
    pr = np.empty(max(m.n_classes, 1), np.int32)
    _check(_lib.nd_motif_export_lambda(m.handle, lam.ctypes.data, pr.ctypes.data), "nd_motif_export_lambda")
    return (lam[:m.n_classes], pr[:m.n_classes]) if paired else lam[:m.n_classes]


# ------------------------------------------------------------------ moments
def nd_make_probes(g: Graph, motifs, n_probes: int, seed: int, flags: int, Z, stream=None):
    import torch
    dt = torch.float64 if flags & ND_STATE_FP64 else torch.float32
    pz = _dev(Z, dt, g.n * n_probes, "Z")
    _check(_lib.nd_make_probes(g.handle, _h(motifs), n_probes, seed, flags, pz, _stream(stream)), "nd_make_probes")


def nd_cheb_moments(g: Graph, motifs, n_probes: int, n_moments: int, seed: int, flags: int, mu,
                    mu_pp=None, stream=None):
    import torch
    pm = _dev(mu, torch.float64, n_moments, "mu")
    pp = _dev(mu_pp, torch.float64, n_probes * n_moments, "mu_pp")
    _check(_lib.nd_cheb_moments(g.handle, _h(motifs), n_probes, n_moments, seed, flags, pm, pp, _stream(stream)),
           "nd_cheb_moments")


def nd_cheb_moments_noalloc(g: Graph, n_probes: int, n_moments: int, seed: int, flags: int, mu, mu_pp=None,
                            stream=None):
    """nd_cheb_moments on the library's fixed device workspace (no allocation)."""
    import torch
    pm = _dev(mu, torch.float64, n_moments, "mu")
    pp = _dev(mu_pp, torch.float64, n_probes * n_moments, "mu_pp")
    _check(_lib.nd_cheb_moments_noalloc(g.handle, n_probes, n_moments, seed, flags, pm, pp, _stream(stream)),
           "nd_cheb_moments_noalloc")


def nd_ldos_moments(g: Graph, motifs, n_probes: int, n_moments: int, seed: int, flags: int, ldos,
                    cv_g=None, ldos_sq=None, mu=None, stream=None):
    import torch
    nm = g.n * n_moments
    pl = _dev(ldos, torch.float64, nm, "ldos")
    pg = _dev(cv_g, torch.float32, nm, "cv_g")
    ps = _dev(ldos_sq, torch.float64, nm, "ldos_sq")
    pm = _dev(mu, torch.float64, n_moments, "mu")
    _check(_lib.nd_ldos_moments(g.handle, _h(motifs), n_probes, n_moments, seed, flags, pg, pl, ps, pm,
                                _stream(stream)), "nd_ldos_moments")


def nd_pdos_nodes(g: Graph, nodes, n_moments: int, flags: int, pdos, stream=None):
    """Exact PDOS moments of the nodes in the device int32 tensor `nodes`."""
    import torch
    n = int(nodes.numel()) if nodes is not None else 0
    pn = _dev(nodes, torch.int32, n, "nodes")
    pp = _dev(pdos, torch.float64, n * n_moments, "pdos")
    _check(_lib.nd_pdos_nodes(g.handle, pn, n, n_moments, flags, pp, _stream(stream)), "nd_pdos_nodes")


def nd_pdos_nested(g: Graph, n_moments: int, pdos, leaf_size: int = 64, max_entries: int = 1 << 30,
                   flags: int = 0, stream=None) -> dict:
    """Exact PDOS moments of all nodes by nested dissection; returns the
    partition statistics."""
    import torch
    pp = _dev(pdos, torch.float64, g.n * n_moments, "pdos")
    st = np.zeros(4, np.int64)
    _check(_lib.nd_pdos_nested(g.handle, n_moments, leaf_size, max_entries, flags, pp, st.ctypes.data,
                               _stream(stream)), "nd_pdos_nested")
    return {"tree_nodes": int(st[0]), "depth": int(st[1]), "separator_nodes": int(st[2]), "block_entries": int(st[3])}


def nd_nested_tree(row_ptr, col, n: int, leaf_size: int = 64) -> dict:
    """The nested-dissection tree of a host CSR graph (no device work):
    owner [n] (tree node of each node's separator), parent [tree nodes] and
    the partition statistics."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    if rp.size != n + 1 or cl.size != int(rp[-1]):
        raise ValueError("row_ptr / col sizes do not match n")
    owner = np.full(n, -1, np.int32)
    parent = np.full(2 * n, -2, np.int32)
    st = np.zeros(4, np.int64)
    _check(_lib.nd_nested_tree(rp.ctypes.data, cl.ctypes.data if cl.size else None, n, leaf_size,
                               owner.ctypes.data, parent.ctypes.data, st.ctypes.data), "nd_nested_tree")
    T = int(st[0])
    return {"owner": owner, "parent": parent[:T].copy(), "tree_nodes": T, "depth": int(st[1]),
            "separator_nodes": int(st[2]), "block_entries": int(st[3])}


def nd_gql(g: Graph, motifs, n_probes: int, n_steps: int, seed: int, flags: int, nodes, weights, steps=None,
           alpha=None, beta=None, stream=None):
    import torch
    kk = n_probes * n_steps
    pn = _dev(nodes, torch.float64, kk, "nodes")
    pw = _dev(weights, torch.float64, kk, "weights")
    ps = _dev(steps, torch.int32, n_probes, "steps")
    pa = _dev(alpha, torch.float64, kk, "alpha")
    pb = _dev(beta, torch.float64, kk, "beta")
    _check(_lib.nd_gql(g.handle, _h(motifs), n_probes, n_steps, seed, flags, pn, pw, ps, pa, pb, _stream(stream)),
           "nd_gql")


def nd_gql_pdos(g: Graph, vertices, n_steps: int, flags: int, nodes, weights, steps=None, stream=None):
    """Gauss rules of the PDOS of the nodes in the device int32 tensor `vertices`."""
    import torch
    nv = int(vertices.numel())
    pv = _dev(vertices, torch.int32, nv, "vertices")
    pn = _dev(nodes, torch.float64, nv * n_steps, "nodes")
    pw = _dev(weights, torch.float64, nv * n_steps, "weights")
    ps = _dev(steps, torch.int32, nv, "steps")
    _check(_lib.nd_gql_pdos(g.handle, pv, nv, n_steps, flags, pn, pw, ps, _stream(stream)), "nd_gql_pdos")


def nd_gql_density(nodes, weights, n_probes: int, n_steps: int, n_moments: int = 0, mu=None, n_bins: int = 0,
                   lo: float = -1.0, hi: float = 1.0, hist=None, stream=None):
    import torch
    kk = n_probes * n_steps
    pn = _dev(nodes, torch.float64, kk, "nodes")
    pw = _dev(weights, torch.float64, kk, "weights")
    pm = _dev(mu, torch.float64, n_moments, "mu") if mu is not None else None
    ph = _dev(hist, torch.float64, n_bins, "hist") if hist is not None else None
    _check(_lib.nd_gql_density(pn, pw, n_probes, n_steps, n_moments, pm, n_bins, lo, hi, ph, _stream(stream)),
           "nd_gql_density")


def nd_reconstruct(mu, n_rows: int, n_moments: int, kernel: int = ND_KERNEL_JACKSON, spikes=(),
                   n_bins: int = 0, lo: float = -1.0, hi: float = 1.0, hist=None, n_points: int = 0,
                   rho=None, stream=None):
    import torch
    pm = _dev(mu, torch.float64, n_rows * n_moments, "mu")
    ph = _dev(hist, torch.float64, n_rows * n_bins, "hist") if hist is not None else None
    pr = _dev(rho, torch.float64, n_rows * n_points, "rho") if rho is not None else None
    lam = np.array([s[0] for s in spikes], np.float64)
    w = np.array([s[1] for s in spikes], np.float64)
    _check(_lib.nd_reconstruct(pm, n_rows, n_moments, kernel, lam.ctypes.data if len(spikes) else None,
                               w.ctypes.data if len(spikes) else None, len(spikes), n_bins, lo, hi, ph,
                               n_points, pr, _stream(stream)), "nd_reconstruct")


# ------------------------------------------------------------------ learned control variate
N_FEAT, WIDTH = 5, 128


def n_params(n_out: int) -> int:
    return N_FEAT * WIDTH + WIDTH + WIDTH * WIDTH + WIDTH + WIDTH * n_out + n_out


def nd_node_features(g: Graph, feat, mean=None, std=None, stream=None):
    import torch
    _check(_lib.nd_node_features(g.handle, _dev(mean, torch.float32, N_FEAT, "mean"),
                                 _dev(std, torch.float32, N_FEAT, "std"), _dev(feat, torch.float32, g.n * N_FEAT, "feat"),
                                 _stream(stream)), "nd_node_features")


def nd_cv_exact_diag(g: Graph, cv_g, ld: int, n_cols: int = 4, stream=None):
    """Overwrite columns 0..n_cols-1 of cv_g [N][ld] with the exact T_m(H)_ii."""
    import torch
    _check(_lib.nd_cv_exact_diag(g.handle, _dev(cv_g, torch.float32, g.n * ld, "cv_g"), ld, n_cols,
                                 _stream(stream)), "nd_cv_exact_diag")


def nd_motif_diag(m: Motifs, cv_g, ld: int, n_cols: int, scale: float = 1.0, stream=None):
    """cv_g [N][ld] += scale (1 - 1/|C|) T_m(lambda_C) for class members, m < n_cols."""
    import torch
    _check(_lib.nd_motif_diag(m.handle, _dev(cv_g, torch.float32, m.graph.n * ld, "cv_g"), ld, n_cols,
                              float(scale), _stream(stream)), "nd_motif_diag")


def nd_ldos_variance(ldos, ldos_sq, n: int, n_moments: int, m_lo: int, n_probes: int, out, per_m=None,
                     stream=None):
    import torch
    _check(_lib.nd_ldos_variance(_dev(ldos, torch.float64, n * n_moments, "ldos"),
                                 _dev(ldos_sq, torch.float64, n * n_moments, "ldos_sq"), n, n_moments, m_lo,
                                 n_probes, _dev(out, torch.float64, 1, "out"),
                                 _dev(per_m, torch.float64, n_moments, "per_m"), _stream(stream)),
           "nd_ldos_variance")


def nd_column_stats(x, n_rows: int, n_cols: int, mean, std, stream=None):
    import torch
    _check(_lib.nd_column_stats(_dev(x, torch.float32, n_rows * n_cols, "x"), n_rows, n_cols,
                                _dev(mean, torch.float32, n_cols, "mean"), _dev(std, torch.float32, n_cols, "std"),
                                _stream(stream)), "nd_column_stats")


def nd_mlp_forward(params, feat, n: int, n_out: int, g, stream=None):
    import torch
    _check(_lib.nd_mlp_forward(_dev(params, torch.float32, n_params(n_out), "params"),
                               _dev(feat, torch.float32, n * N_FEAT, "feat"), n, n_out,
                               _dev(g, torch.float32, n * n_out, "g"), _stream(stream)), "nd_mlp_forward")


def nd_mlp_grad(params, feat, target, ld_target: int, idx, n: int, n_out: int, grad, loss, stream=None):
    import torch
    rows = feat.numel() // N_FEAT
    if idx is not None:
        pidx = _dev(idx, torch.int32, n, "idx")
    else:
        pidx = None
        if rows < n:
            raise ValueError("feat holds %d rows, needs %d" % (rows, n))
    if target.numel() < rows * ld_target or ld_target < n_out:
        raise ValueError("target too small for ld_target=%d" % ld_target)
    _check(_lib.nd_mlp_grad(_dev(params, torch.float32, n_params(n_out), "params"),
                            _dev(feat, torch.float32, rows * N_FEAT, "feat"),
                            _dev(target, torch.float32, rows * ld_target, "target"), ld_target, pidx, n, n_out,
                            _dev(grad, torch.float32, n_params(n_out), "grad"), _dev(loss, torch.float32, 1, "loss"),
                            _stream(stream)), "nd_mlp_grad")


def nd_adam_step(params, m, v, grad, n_params_: int, t: int, lr: float, stream=None):
    import torch
    _check(_lib.nd_adam_step(_dev(params, torch.float32, n_params_, "params"), _dev(m, torch.float32, n_params_, "m"),
                             _dev(v, torch.float32, n_params_, "v"), _dev(grad, torch.float32, n_params_, "grad"),
                             n_params_, t, lr, _stream(stream)), "nd_adam_step")
