"""MI355X matrix-P Gaussian-boson-sampling hot path (arXiv:2503.12749).

Thin Python layer over libmpgbs.so (include/mpgbs.h).  The functions below
keep the C entry-point names and only marshal arguments: every step of the
path (sampling, propagation, occupations, characteristic function, sample
reduction, inverse DFT) runs in the library's HIP kernels.  PyTorch provides
device memory and the stream.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import BIN_MODES, ESTIMATORS, MPError, PRECISIONS, i32_array

__all__ = [
    "mp_ld_modes", "mp_ab_bytes", "mp_c_bytes", "mp_sample", "mp_propagate_workspace",
    "mp_propagate", "mp_pack_transmission", "mp_propagate_packed", "mp_occupations",
    "mp_moments_accumulate", "mp_observable_histogram", "mp_subensemble_stats", "mp_acc_entries",
    "mp_binned_workspace", "mp_binned_counts", "mp_counts_finalize", "mp_finalize_workspace",
    "mp_mode_occupations_bytes", "mp_mode_occupations", "mp_pair_correlations_accumulate",
    "mp_pair_correlations_workspace", "mp_propagate_counts_workspace", "mp_propagate_counts", "mp_propagate_counts_noalloc",
    "mp_version", "CountsPipeline",
    "PairPipeline", "Plan", "MPError", "mp_check_finite", "mp_mfma_sustained",
]


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _mode(m) -> int:
    return BIN_MODES[m] if isinstance(m, str) else int(m)


def _est(e) -> int:
    return ESTIMATORS[e] if isinstance(e, str) else int(e)


def mp_ld_modes(M: int) -> int:
    return int(_lib.load().mp_ld_modes(M))


def mp_ab_bytes(M: int, E: int, prec) -> int:
    return int(_lib.load().mp_ab_bytes(M, E, _prec(prec)))


def mp_c_bytes(M: int, E: int, prec) -> int:
    return int(_lib.load().mp_c_bytes(M, E, _prec(prec)))


def mp_propagate_workspace(M: int, prec) -> int:
    return int(_lib.load().mp_propagate_workspace(M, _prec(prec)))


def mp_acc_entries(d: int, mode, K) -> int:
    return int(_lib.load().mp_acc_entries(d, _mode(mode), i32_array(K)))


def mp_binned_workspace(d: int, mode, K, E: int, n_sub: int, samples_per_sub: int, e0: int) -> int:
    return int(_lib.load().mp_binned_workspace(d, _mode(mode), i32_array(K), E, n_sub,
                                               samples_per_sub, e0))


def mp_version() -> str:
    return _lib.load().mp_version().decode()


def mp_sample(M, g0, E, r, seed, net, prec, ab, n_out, stream=None):
    """r: device float64[M]; ab: device buffer of mp_ab_bytes; n_out: device float64[E]."""
    _lib.check(_lib.load().mp_sample(M, g0, E, _ptr(r), seed, net, _prec(prec), _ptr(ab),
                                     _ptr(n_out), _stream(stream)))


def mp_propagate(M, E, T, prec, ab, C, workspace, stream=None):
    """T: device float64 view of the row-major complex M x M matrix."""
    _lib.check(_lib.load().mp_propagate(M, E, _ptr(T), _prec(prec), _ptr(ab), _ptr(C),
                                        _ptr(workspace), workspace.numel() * workspace.element_size(),
                                        _stream(stream)))


def mp_pack_transmission(M, T, prec, workspace, stream=None):
    nbytes = workspace.numel() * workspace.element_size()
    _lib.check(_lib.load().mp_pack_transmission(M, _ptr(T), _prec(prec), _ptr(workspace), nbytes,
                                                _stream(stream)))


def mp_propagate_packed(M, E, prec, ab, C, workspace, stream=None):
    nbytes = workspace.numel() * workspace.element_size()
    _lib.check(_lib.load().mp_propagate_packed(M, E, _prec(prec), _ptr(ab), _ptr(C),
                                               _ptr(workspace), nbytes, _stream(stream)))


def mp_binned_counts(M, E, C, n, prec, est, d, bin_of_mode, mode, m_lo, K, n_sub,
                     samples_per_sub, e0, acc, workspace, stream=None):
    """bin_of_mode, m_lo, K: host integer sequences."""
    _lib.check(_lib.load().mp_binned_counts(
        M, E, _ptr(C), _ptr(n), _prec(prec), _est(est), d, i32_array(bin_of_mode), _mode(mode),
        i32_array(m_lo), i32_array(K), n_sub, samples_per_sub, e0, _ptr(acc), _ptr(workspace),
        workspace.numel() * workspace.element_size(), _stream(stream)))


def mp_occupations(M, E, C, prec, d, bin_of_mode, mode, nq, stream=None):
    """bin_of_mode: host integer sequence; nq: device float64 (E * n_dist * 2)."""
    _lib.check(_lib.load().mp_occupations(M, E, _ptr(C), _prec(prec), d, i32_array(bin_of_mode),
                                          _mode(mode), _ptr(nq), _stream(stream)))


def mp_moments_accumulate(E, n, nq, n_dist, kmax, est, n_sub, samples_per_sub, e0, acc,
                          stream=None):
    _lib.check(_lib.load().mp_moments_accumulate(E, _ptr(n), _ptr(nq), n_dist, kmax, _est(est),
                                                 n_sub, samples_per_sub, e0, _ptr(acc),
                                                 _stream(stream)))


def mp_observable_histogram(E, n, nq, n_dist, q, m, est, o_min, width, n_bins, n_sub,
                            samples_per_sub, e0, hist, stream=None):
    _lib.check(_lib.load().mp_observable_histogram(E, _ptr(n), _ptr(nq), n_dist, q, m, _est(est),
                                                   float(o_min), float(width), n_bins, n_sub,
                                                   samples_per_sub, e0, _ptr(hist),
                                                   _stream(stream)))


def mp_subensemble_stats(n_sub, samples_per_sub, n_vals, ncomp, scale, acc, mean, sigma,
                         stream=None):
    _lib.check(_lib.load().mp_subensemble_stats(n_sub, samples_per_sub, n_vals, ncomp,
                                                float(scale), _ptr(acc), _ptr(mean), _ptr(sigma),
                                                _stream(stream)))


def mp_check_finite(x, scratch, stream=None) -> int:
    """Synchronous: raises MPError (MP_ERR_NONFINITE) if the device float64
    tensor x holds NaN or infinite values; scratch is a device tensor of at
    least 8 bytes.  Returns the count of such values (0)."""
    bad = ctypes.c_int64(0)
    _lib.check(_lib.load().mp_check_finite(_ptr(x), x.numel(), _ptr(scratch), ctypes.byref(bad),
                                           _stream(stream)))
    return bad.value


def mp_mfma_sustained(kind: int, iters: int, sink, stream=None) -> float:
    """Launches the matrix-core rate probe (kind 0: FP16 32x32x16, 1: FP32
    32x32x2, 2: FP64 16x16x4) on `stream`; sink is a device float64 tensor of
    at least 256 entries per compute unit.  Returns the launch's flop count."""
    flops = ctypes.c_double(0.0)
    _lib.check(_lib.load().mp_mfma_sustained(kind, iters, _ptr(sink), sink.numel() * 8,
                                             ctypes.byref(flops), _stream(stream)))
    return flops.value


def mp_mode_occupations_bytes(M: int, E: int, prec) -> int:
    return int(_lib.load().mp_mode_occupations_bytes(M, E, _prec(prec)))


def mp_mode_occupations(M, E, C, prec, X, stream=None):
    _lib.check(_lib.load().mp_mode_occupations(M, E, _ptr(C), _prec(prec), _ptr(X),
                                               _stream(stream)))


def mp_pair_correlations_workspace(M, E, prec, samples_per_sub, e0) -> int:
    return int(_lib.load().mp_pair_correlations_workspace(M, E, _prec(prec), samples_per_sub, e0))


def mp_pair_correlations_accumulate(M, E, X, prec, n_sub, samples_per_sub, e0, acc,
                                    workspace=None, stream=None):
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _lib.check(_lib.load().mp_pair_correlations_accumulate(M, E, _ptr(X), _prec(prec), n_sub,
                                                           samples_per_sub, e0, _ptr(acc),
                                                           _ptr(workspace), nbytes,
                                                           _stream(stream)))


def mp_propagate_counts_workspace(M, E, d, bin_of_mode, mode, K, n_sub, samples_per_sub, e0):
    return int(_lib.load().mp_propagate_counts_workspace(M, E, d, i32_array(bin_of_mode), _mode(mode),
                                                         i32_array(K), n_sub, samples_per_sub, e0))


def mp_propagate_counts(M, E, prec, est, ab, n, packed, d, bin_of_mode, mode, m_lo, K, n_sub,
                        samples_per_sub, e0, acc, workspace, stream=None):
    """Occupation-fused propagate + counts; bin_of_mode, m_lo, K: host sequences."""
    _lib.check(_lib.load().mp_propagate_counts(
        M, E, _prec(prec), _est(est), _ptr(ab), _ptr(n), _ptr(packed),
        packed.numel() * packed.element_size(), d, i32_array(bin_of_mode), _mode(mode),
        i32_array(m_lo), i32_array(K), n_sub, samples_per_sub, e0, _ptr(acc), _ptr(workspace),
        workspace.numel() * workspace.element_size(), _stream(stream)))


def mp_bilinear_workspace(M) -> int:
    return int(_lib.load().mp_bilinear_workspace(M))


def mp_bilinear_packed_bytes(M) -> int:
    return int(_lib.load().mp_bilinear_packed_bytes(M))


def mp_pack_bilinear(M, T, bin_of_mode, prec, packed, scratch, stream=None):
    """W = T^T P_S T* (S: modes with bin_of_mode == 0) packed as prec packs T;
    T is the device complex128 operand (as a float64 tensor), bin_of_mode a
    host sequence of 0 / -1."""
    _lib.check(_lib.load().mp_pack_bilinear(
        M, _ptr(T), i32_array(bin_of_mode), _prec(prec), _ptr(packed),
        packed.numel() * packed.element_size(), _ptr(scratch),
        scratch.numel() * scratch.element_size(), _stream(stream)))


def mp_propagate_counts_bilinear(M, E, prec, est, ab, n, packed, m_lo, K, n_sub, samples_per_sub,
                                 e0, acc, workspace, stream=None):
    """One distribution through the bilinear form alpha^T W beta; m_lo, K: ints."""
    _lib.check(_lib.load().mp_propagate_counts_bilinear(
        M, E, _prec(prec), _est(est), _ptr(ab), _ptr(n), _ptr(packed),
        packed.numel() * packed.element_size(), i32_array([m_lo]), i32_array([K]), n_sub,
        samples_per_sub, e0, _ptr(acc), _ptr(workspace),
        workspace.numel() * workspace.element_size(), _stream(stream)))


def mp_propagate_counts_noalloc(M, E, prec, est, ab, n, packed, d, bin_of_mode, mode, m_lo, K,
                                n_sub, samples_per_sub, e0, acc, stream=None):
    """mp_propagate_counts on the library's own device scratch (no workspace
    argument, nothing allocated); bin_of_mode, m_lo, K: host sequences."""
    _lib.check(_lib.load().mp_propagate_counts_noalloc(
        M, E, _prec(prec), _est(est), _ptr(ab), _ptr(n), _ptr(packed),
        packed.numel() * packed.element_size(), d, i32_array(bin_of_mode), _mode(mode),
        i32_array(m_lo), i32_array(K), n_sub, samples_per_sub, e0, _ptr(acc), _stream(stream)))


def mp_finalize_workspace(d: int, mode, K, n_sub: int) -> int:
    return int(_lib.load().mp_finalize_workspace(d, _mode(mode), i32_array(K), n_sub))


def mp_counts_finalize(d, mode, K, n_sub, samples_per_sub, acc, P_re, P_im, sigma, workspace=None,
                       stream=None):
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _lib.check(_lib.load().mp_counts_finalize(d, _mode(mode), i32_array(K), n_sub, samples_per_sub,
                                              _ptr(acc), _ptr(P_re), _ptr(P_im), _ptr(sigma),
                                              _ptr(workspace), nbytes, _stream(stream)))


class CountsPipeline:
    """Owns the device buffers of one workload and runs it chunk by chunk:
    mp_sample -> mp_propagate_packed -> mp_binned_counts per chunk, then
    mp_counts_finalize.  All buffers are allocated once, in __init__, and T is
    packed once, on the first chunk after construction."""

    def __init__(self, T: np.ndarray, r: np.ndarray, *, prec="fp64", seed: int, net: int = 0,
                 bin_of_mode=None, d: int = 1, mode="joint", windows, n_sub: int,
                 samples_per_sub: int, chunk: int, est="matrix_p", device="cuda:0",
                 fused: bool = False, bilinear: bool = False):
        import torch
        self.torch = torch
        T = np.ascontiguousarray(T, dtype=np.complex128)
        self.M = int(T.shape[0])
        assert T.shape == (self.M, self.M)
        self.prec = _prec(prec)
        self.est = _est(est)
        self.mode = _mode(mode)
        self.seed, self.net, self.d = int(seed), int(net), int(d)
        self.bins = (np.zeros(self.M, np.int32) if bin_of_mode is None
                     else np.asarray(bin_of_mode, dtype=np.int32))
        self.m_lo = [int(w[0]) for w in windows]
        self.K = [int(w[1]) for w in windows]
        self.n_sub, self.ns, self.chunk = int(n_sub), int(samples_per_sub), int(chunk)
        dev = torch.device(device)
        self.device = dev
        self.T = torch.from_numpy(T.view(np.float64).reshape(-1).copy()).to(dev)
        self.r = torch.from_numpy(np.asarray(r, dtype=np.float64).copy()).to(dev)
        self.fused = bool(fused) or bool(bilinear)
        # one distribution through alpha^T W beta, W = T^T P_S T* formed once
        # (mp_pack_bilinear) in place of packing T
        self.bilinear = bool(bilinear)
        if self.bilinear and not (self.d == 1 and self.prec == _lib.PRECISIONS["split1t_f8"]):
            raise MPError(-4, "the bilinear form takes one distribution (d = 1) in split1t_f8")
        self.ab = torch.empty(mp_ab_bytes(self.M, self.chunk, self.prec), dtype=torch.uint8, device=dev)
        # the occupation-fused path never materialises C
        self.C = None if self.fused else torch.empty(mp_c_bytes(self.M, self.chunk, self.prec),
                                                      dtype=torch.uint8, device=dev)
        self.n = torch.empty(self.chunk, dtype=torch.float64, device=dev)
        pbytes = (mp_bilinear_packed_bytes(self.M) if self.bilinear
                  else mp_propagate_workspace(self.M, self.prec))
        self.ws_prop = torch.empty(pbytes, dtype=torch.uint8, device=dev)
        self.packed = False
        self.entries = mp_acc_entries(self.d, self.mode, self.K)
        if self.entries < 0:
            raise MPError(-1, "invalid bin layout")
        # a chunk touches at most chunk // ns + 2 sub-ensembles, each adding at
        # most one partial tile of 64 samples
        blocks = -(-self.chunk // 64) + self.chunk // self.ns + 2
        wbytes = blocks * self.entries * 16 + 256
        if self.mode == 0 and self.d >= 2:
            wbytes = mp_binned_workspace(self.d, 0, self.K, self.chunk, self.n_sub, self.ns, 0)
        if self.fused:
            # the GEMM's partials plus the counts blocks of the worst chunk alignment (the
            # bilinear form's partials cover one run of all modes)
            wbins = np.zeros(self.M, np.int32) if self.bilinear else self.bins
            wbytes += mp_propagate_counts_workspace(self.M, self.chunk, self.d, wbins, self.mode,
                                                    self.K, self.n_sub, self.ns, 0)
        self.ws_counts = torch.empty(wbytes, dtype=torch.uint8, device=dev)
        self.acc = torch.zeros(self.n_sub * self.entries * 2, dtype=torch.float64, device=dev)
        self.P_re = torch.empty(self.entries, dtype=torch.float64, device=dev)
        self.P_im = torch.empty(self.entries, dtype=torch.float64, device=dev)
        self.sigma = torch.empty(self.entries, dtype=torch.float64, device=dev)
        fw = mp_finalize_workspace(self.d, self.mode, self.K, self.n_sub)
        self.ws_final = torch.empty(fw, dtype=torch.uint8, device=dev) if fw else None

    def reset(self):
        self.acc.zero_()

    def run_chunk(self, g0: int, E: int, stream=None):
        assert 1 <= E <= self.chunk
        if not self.packed:
            if self.bilinear:
                scratch = self.torch.empty(mp_bilinear_workspace(self.M), dtype=self.torch.uint8,
                                           device=self.device)
                mp_pack_bilinear(self.M, self.T, self.bins, self.prec, self.ws_prop, scratch, stream)
                self.torch.cuda.synchronize()  # once per run: the scratch is free to go
                del scratch
            else:
                mp_pack_transmission(self.M, self.T, self.prec, self.ws_prop, stream)
            self.packed = True
        mp_sample(self.M, g0, E, self.r, self.seed, self.net, self.prec, self.ab, self.n, stream)
        if self.bilinear:
            mp_propagate_counts_bilinear(self.M, E, self.prec, self.est, self.ab, self.n,
                                         self.ws_prop, self.m_lo[0], self.K[0], self.n_sub, self.ns,
                                         g0, self.acc, self.ws_counts, stream)
            return
        if self.fused:
            mp_propagate_counts(self.M, E, self.prec, self.est, self.ab, self.n, self.ws_prop, self.d,
                                self.bins, self.mode, self.m_lo, self.K, self.n_sub, self.ns, g0,
                                self.acc, self.ws_counts, stream)
            return
        mp_propagate_packed(self.M, E, self.prec, self.ab, self.C, self.ws_prop, stream)
        self.counts_chunk(g0, E, stream)

    def counts_chunk(self, g0: int, E: int, stream=None):
        mp_binned_counts(self.M, E, self.C, self.n, self.prec, self.est, self.d, self.bins, self.mode,
                         self.m_lo, self.K, self.n_sub, self.ns, g0, self.acc, self.ws_counts, stream)

    def finalize(self, stream=None):
        mp_counts_finalize(self.d, self.mode, self.K, self.n_sub, self.ns, self.acc, self.P_re,
                           self.P_im, self.sigma, self.ws_final, stream)

    def run(self, E_total: int | None = None, g_start: int = 0, stream=None):
        E_total = self.n_sub * self.ns if E_total is None else E_total
        done = 0
        while done < E_total:
            c = min(self.chunk, E_total - done)
            self.run_chunk(g_start + done, c, stream)
            done += c
        self.finalize(stream)

    def checkpoint(self, next_g: int) -> dict:
        """What a run needs to continue after its last chunk: a host copy of the
        per-sub-ensemble FP64 accumulators and the next global sample index
        (synchronises).  The noise is counter-based, so a run restored from it
        and continued with the same chunk boundaries equals the uninterrupted
        run bit for bit."""
        return {"acc": self.acc.cpu().numpy().copy(), "next_g": int(next_g)}

    def restore(self, state: dict) -> int:
        """Loads accumulators saved by checkpoint(); returns the next sample
        index, from which run(E_total - next_g, g_start=next_g) continues."""
        a = np.ascontiguousarray(state["acc"], dtype=np.float64).reshape(-1)
        if a.size != self.acc.numel():
            raise ValueError(f"checkpoint holds {a.size} accumulator values, this pipeline "
                             f"{self.acc.numel()}")
        self.acc.copy_(self.torch.from_numpy(a).to(self.acc.device))
        return int(state["next_g"])

    def result(self):
        """(P_re, P_im, sigma) as numpy arrays (synchronises); raises MPError
        (MP_ERR_NONFINITE) if the estimate holds NaN or infinite values."""
        scratch = self.torch.empty(1, dtype=self.torch.int64, device=self.P_re.device)
        mp_check_finite(self.P_re, scratch)
        mp_check_finite(self.P_im, scratch)
        return (self.P_re.cpu().numpy(), self.P_im.cpu().numpy(), self.sigma.cpu().numpy())

    def alpha_beta(self, E: int):
        """Views of the last chunk's stored amplitudes as numpy (E, M) arrays
        (FP64, FP32 and the single FP16 storage of the two T-split forms;
        synchronises)."""
        t = self.torch
        ldm = mp_ld_modes(self.M)
        if self.prec in (_lib.PRECISIONS["split1t_fp16"], _lib.PRECISIONS["split1t_f8"]):
            h = self.ab.view(t.float16).double().cpu().numpy()
            e2 = E + (E & 1)
            j = np.arange(self.M)
            def cols(c):
                c = np.asarray(c)[:, None]
                return h[(c >> 1) * 2 * ldm + 64 * (j >> 5) + (j & 31) + (c & 1) * 32]
            return cols(np.arange(E)), cols(e2 + np.arange(E))
        dt = {0: t.float64, 1: t.float32}[self.prec]
        v = self.ab.view(dt)[: ldm * 2 * E].reshape(2 * E, ldm)[:, : self.M].double().cpu().numpy()
        return v[:E], v[E:]

    def propagated(self, E: int):
        """(alpha', beta') of the last chunk as complex numpy (E, M) arrays."""
        t = self.torch
        ldm = mp_ld_modes(self.M)
        dt = t.float64 if self.prec == 0 else t.float32
        v = self.C.view(dt)[: 2 * ldm * 2 * E].reshape(2 * E, 2 * ldm).double().cpu().numpy()
        a = v[:E, : self.M] + 1j * v[:E, ldm: ldm + self.M]
        b = v[E:, : self.M] - 1j * v[E:, ldm: ldm + self.M]
        return a, b


class PairPipeline:
    """Normally ordered pair moments <:n_i n_j:> of all output modes from one
    ensemble: per chunk mp_sample -> mp_propagate_packed -> mp_mode_occupations
    -> mp_pair_correlations_accumulate, then mp_subensemble_stats.  Buffers
    are allocated once; T is packed on the first chunk."""

    def __init__(self, T: np.ndarray, r: np.ndarray, *, prec="fp32", seed: int, net: int = 0,
                 n_sub: int, samples_per_sub: int, chunk: int, device="cuda:0"):
        import torch
        self.torch = torch
        T = np.ascontiguousarray(T, dtype=np.complex128)
        self.M = int(T.shape[0])
        assert T.shape == (self.M, self.M)
        self.prec = _prec(prec)
        self.seed, self.net = int(seed), int(net)
        self.n_sub, self.ns, self.chunk = int(n_sub), int(samples_per_sub), int(chunk)
        dev = torch.device(device)
        self.T = torch.from_numpy(T.view(np.float64).reshape(-1).copy()).to(dev)
        self.r = torch.from_numpy(np.asarray(r, dtype=np.float64).copy()).to(dev)
        self.ab = torch.empty(mp_ab_bytes(self.M, self.chunk, self.prec), dtype=torch.uint8, device=dev)
        self.C = torch.empty(mp_c_bytes(self.M, self.chunk, self.prec), dtype=torch.uint8, device=dev)
        self.n = torch.empty(self.chunk, dtype=torch.float64, device=dev)
        self.ws_prop = torch.empty(mp_propagate_workspace(self.M, self.prec), dtype=torch.uint8,
                                   device=dev)
        self.X = torch.empty(mp_mode_occupations_bytes(self.M, self.chunk, self.prec),
                             dtype=torch.uint8, device=dev)
        nv = self.M * self.M
        self.acc = torch.zeros(self.n_sub * nv * 2, dtype=torch.float64, device=dev)
        self.ws = torch.empty(256, dtype=torch.uint8, device=dev)
        self.mean = torch.empty(nv * 2, dtype=torch.float64, device=dev)
        self.sigma = torch.empty(nv, dtype=torch.float64, device=dev)
        self.packed = False

    def run_chunk(self, g0: int, E: int, stream=None):
        assert 1 <= E <= self.chunk
        if not self.packed:
            mp_pack_transmission(self.M, self.T, self.prec, self.ws_prop, stream)
            self.packed = True
        mp_sample(self.M, g0, E, self.r, self.seed, self.net, self.prec, self.ab, self.n, stream)
        mp_propagate_packed(self.M, E, self.prec, self.ab, self.C, self.ws_prop, stream)
        self.pairs_chunk(g0, E, stream)

    def workspace(self, g0: int, E: int):
        """The pair-sum workspace for samples [g0, g0 + E), grown when a
        chunk's alignment or size needs more (a short chunk can need partial
        tiles where a full one does not)."""
        need = mp_pair_correlations_workspace(self.M, E, self.prec, self.ns, g0)
        if need > self.ws.numel():
            self.ws = self.torch.empty(need, dtype=self.torch.uint8, device=self.ws.device)
        return self.ws

    def pairs_chunk(self, g0: int, E: int, stream=None):
        mp_mode_occupations(self.M, E, self.C, self.prec, self.X, stream)
        mp_pair_correlations_accumulate(self.M, E, self.X, self.prec, self.n_sub, self.ns, g0,
                                        self.acc, self.workspace(g0, E), stream)

    def finalize(self, stream=None):
        mp_subensemble_stats(self.n_sub, self.ns, self.M * self.M, 2, 1.0, self.acc, self.mean,
                             self.sigma, stream)

    def run(self, E_total: int | None = None, g_start: int = 0, stream=None):
        E_total = self.n_sub * self.ns if E_total is None else E_total
        done = 0
        while done < E_total:
            c = min(self.chunk, E_total - done)
            self.run_chunk(g_start + done, c, stream)
            done += c
        self.finalize(stream)

    def result(self):
        """(G2, sigma): complex (M, M) means and sigma_T of their real parts
        (synchronises); raises MPError (MP_ERR_NONFINITE) if the means hold
        NaN or infinite values."""
        scratch = self.torch.empty(1, dtype=self.torch.int64, device=self.mean.device)
        mp_check_finite(self.mean, scratch)
        m = self.mean.cpu().numpy().view(np.complex128).reshape(self.M, self.M)
        return m, self.sigma.cpu().numpy().reshape(self.M, self.M)

    def subensemble_sums(self):
        """Per sub-ensemble sums, complex (n_sub, M, M) (synchronises)."""
        return self.acc.cpu().numpy().view(np.complex128).reshape(self.n_sub, self.M, self.M)


_HIP = None


def _hip_runtime():
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _HIP.hipMemcpy.restype = ctypes.c_int
    return _HIP


class Plan:
    """Batched plan over many networks (mp_plan_create / mp_plan_launch):
    one captured hipGraph per plan, one persistent grouped GEMM launch with
    the occupation-fused epilogue per pass (split precisions).  `nets` is a
    list of dicts with keys T (complex numpy M x M), r, seed, net, E, n_sub
    and either window=(m_lo, K) (the total count of all modes) or
    bin_of_mode, d, mode and windows=[(m_lo, K), ...] (one per distribution,
    as for CountsPipeline)."""

    def __init__(self, nets, *, prec="split_fp16", est="matrix_p", chunk=None, tune_cache=None,
                 device="cuda:0"):
        import torch
        self.torch = torch
        dev = torch.device(device)
        keep = []
        self.K = []  # result entries per network
        descs = (_lib.NetDesc * len(nets))()
        for i, n in enumerate(nets):
            T = np.ascontiguousarray(n["T"], dtype=np.complex128)
            M = T.shape[0]
            Td = torch.from_numpy(T.view(np.float64).reshape(-1).copy()).to(dev)
            rd = torch.from_numpy(np.asarray(n["r"], dtype=np.float64).copy()).to(dev)
            keep += [Td, rd]
            if "windows" in n:  # binned distributions
                d = int(n["d"])
                bins = i32_array(n["bin_of_mode"])
                mlo = i32_array([w[0] for w in n["windows"]])
                Kb = i32_array([w[1] for w in n["windows"]])
                keep += [bins, mlo, Kb]
                descs[i] = _lib.NetDesc(M, Td.data_ptr(), rd.data_ptr(), int(n["seed"]),
                                        int(n["net"]), int(n["E"]), int(n["n_sub"]), 0, 0, d,
                                        _mode(n.get("mode", "joint")),
                                        ctypes.cast(bins, ctypes.c_void_p),
                                        ctypes.cast(mlo, ctypes.c_void_p),
                                        ctypes.cast(Kb, ctypes.c_void_p))
                self.K.append(mp_acc_entries(d, n.get("mode", "joint"),
                                             [w[1] for w in n["windows"]]))
            else:
                m_lo, K = n["window"]
                descs[i] = _lib.NetDesc(M, Td.data_ptr(), rd.data_ptr(), int(n["seed"]),
                                        int(n["net"]), int(n["E"]), int(n["n_sub"]), int(m_lo),
                                        int(K), 0, 0, None, None, None)
                self.K.append(int(K))
        chunk = max(int(n["E"]) for n in nets) if chunk is None else int(chunk)
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        path = None if tune_cache is None else str(tune_cache).encode()
        _lib.check(_lib.load().mp_plan_create(ctypes.byref(h), len(nets), descs, _prec(prec),
                                              _est(est), chunk, path))
        self.handle = h
        self.device = dev
        del keep

    def launch(self, stream=None):
        _lib.check(_lib.load().mp_plan_launch(self.handle, _stream(stream)))

    def result(self, i):
        """(P_re, P_im, sigma) of network i as numpy arrays (synchronises);
        raises MPError (MP_ERR_NONFINITE) if the estimate holds NaN or
        infinite values."""
        t = self.torch
        pr, pi, sg = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        _lib.check(_lib.load().mp_plan_result(self.handle, i, ctypes.byref(pr), ctypes.byref(pi),
                                              ctypes.byref(sg)))
        t.cuda.synchronize()
        K = self.K[i]
        scratch = t.empty(1, dtype=t.int64, device=self.device)
        for ptr in (pr, pi):
            _lib.check(_lib.load().mp_check_finite(ctypes.c_void_p(ptr.value), K, _ptr(scratch),
                                                   None, None))
        out = []
        hip = _hip_runtime()
        for ptr in (pr, pi, sg):
            buf = (ctypes.c_double * K)()
            if hip.hipMemcpy(buf, ctypes.c_void_p(ptr.value), ctypes.c_size_t(8 * K), 2) != 0:
                raise MPError(-3, "hipMemcpy of plan results failed")
            out.append(np.frombuffer(buf, dtype=np.float64).copy())
        return tuple(out)

    def info(self):
        o, f, ms, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double(), ctypes.c_size_t()
        _lib.check(_lib.load().mp_plan_info(self.handle, ctypes.byref(o), ctypes.byref(f),
                                            ctypes.byref(ms), ctypes.byref(b)))
        tiles = []
        for i in range(len(self.K)):
            m, e = ctypes.c_int32(), ctypes.c_int32()
            _lib.check(_lib.load().mp_plan_tile(self.handle, i, ctypes.byref(m), ctypes.byref(e)))
            tiles.append((m.value, e.value))
        return {"order": o.value, "prefetch": f.value, "tuned_ms": ms.value,
                "device_bytes": b.value, "tiles": tiles}

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.check(_lib.load().mp_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
