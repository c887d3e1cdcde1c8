"""Thin ctypes binding of ``libnze.so`` (declared in ``include/nze.h``).

Argument marshalling only: every step of the emulation runs in the library.
PyTorch provides the device workspace and the stream; nothing else.
"""
import atexit
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnze.so")

NZE_OK, NZE_EINVAL, NZE_ENOMEM, NZE_EHIP, NZE_ENOCONV, NZE_EFIT, NZE_ENUM = \
    0, -1, -2, -3, -4, -5, -6
NZE_FP64, NZE_MIXED = 0, 1
NZE_POLY, NZE_EXP3, NZE_LOGLIN_W = 0, 1, 2

c_double_p = ctypes.POINTER(ctypes.c_double)
c_int32_p = ctypes.POINTER(ctypes.c_int32)
c_uint8_p = ctypes.POINTER(ctypes.c_uint8)


class NzeNoise(ctypes.Structure):
    _fields_ = [("dep", ctypes.c_double), ("ad", ctypes.c_double),
                ("px", ctypes.c_double), ("py", ctypes.c_double),
                ("pz", ctypes.c_double)]


class MpoConfig(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("chi_max", ctypes.c_int32),
                ("n_levels", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("trunc_tol", ctypes.c_double), ("tie_tol", ctypes.c_double),
                ("jacobi_tol", ctypes.c_double), ("jacobi_abs", ctypes.c_double),
                ("max_sweeps", ctypes.c_int32), ("block", ctypes.c_int32)]


class NzeStats(ctypes.Structure):
    _fields_ = [("fidelity", ctypes.c_double), ("log_scale", ctypes.c_double),
                ("max_discarded", ctypes.c_double),
                ("min_cut_gap", ctypes.c_double),
                ("max_bond", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("updates", ctypes.c_int64), ("sweeps_total", ctypes.c_int64),
                ("flops", ctypes.c_double), ("cap_hits", ctypes.c_int64),
                ("cap_offdiag", ctypes.c_double), ("ns_scaled", ctypes.c_int64)]


class NzeFitOpts(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int32), ("delta_f", ctypes.c_double),
                ("delta_d", ctypes.c_double), ("small", ctypes.c_double),
                ("dip_threshold", ctypes.c_double),
                ("ref_sign", ctypes.c_int32), ("b_max", ctypes.c_double)]


class NzeTuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("group_scale", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("cross_sweeps", ctypes.c_int32),
                ("cross_min_blocks", ctypes.c_int32),
                ("ms_per_svd", ctypes.c_double)]


class NzeJobSpec(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("chi_max", ctypes.c_int32),
                ("n_levels", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("n_layers", ctypes.c_int32),
                ("layer_gates", ctypes.POINTER(ctypes.c_int32)),
                ("left_sites", ctypes.POINTER(ctypes.c_int32)),
                ("ptm", ctypes.POINTER(ctypes.c_double)),
                ("n_obs", ctypes.c_int32),
                ("paulis", ctypes.POINTER(ctypes.c_uint8))]


class NzeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nze error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "paper_2501_13237_amd.build.build()")
    # torch first: it brings its own HIP runtime, and the library must bind
    # to that same runtime (loaded the other way round, two runtimes open the
    # device and the second finds none)
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    L.nze_build_ptm.argtypes = [c_double_p, c_double_p,
                                ctypes.POINTER(NzeNoise), ctypes.c_double,
                                c_double_p]
    L.nze_build_ptm_pauli.argtypes = [c_double_p, c_double_p, c_double_p,
                                      ctypes.c_double, c_double_p]
    L.nze_ptm_compose_1q.argtypes = [c_double_p, c_double_p, c_double_p,
                                     c_double_p, ctypes.c_double, ctypes.c_int32,
                                     ctypes.c_int32, c_double_p]
    L.nze_ptm_compose.argtypes = [c_double_p, c_double_p, c_double_p]
    L.nze_ptm_swap_qubits.argtypes = [c_double_p, c_double_p]
    L.nze_route_chain.argtypes = [ctypes.c_int32, ctypes.c_int32, c_int32_p, c_int32_p,
                                  ctypes.c_int32, ctypes.c_int32, c_int32_p, c_int32_p,
                                  ctypes.POINTER(ctypes.c_uint8), c_int32_p, c_int32_p]
    L.mpo_footprint.argtypes = [ctypes.POINTER(MpoConfig)]
    L.mpo_footprint.restype = ctypes.c_size_t
    L.mpo_init.argtypes = [ctypes.POINTER(ctypes.c_void_p),
                           ctypes.POINTER(MpoConfig), c_double_p,
                           ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    L.mpo_free.argtypes = [ctypes.c_void_p]
    L.mpo_free.restype = None
    L.mpo_apply_layer.argtypes = [ctypes.c_void_p, ctypes.c_int32, c_int32_p,
                                  c_double_p]
    L.mpo_apply_layer_batch.argtypes = [
        ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, c_int32_p,
        ctypes.POINTER(c_int32_p), ctypes.POINTER(c_double_p)]
    L.mpo_expect.argtypes = [ctypes.c_void_p, ctypes.c_int32, c_uint8_p,
                             c_double_p, c_double_p, c_double_p]
    L.mpo_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(NzeStats),
                            c_int32_p]
    L.mpo_bond_spectrum.argtypes = [ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_int32, c_double_p, ctypes.c_int32,
                                    c_int32_p]
    L.mpo_bond_entropy.argtypes = [ctypes.c_void_p, ctypes.c_int32,
                                   ctypes.c_int32, c_double_p]
    L.mpo_overlap.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                              ctypes.c_int32, c_double_p, c_double_p]
    L.mpo_sync.argtypes = [ctypes.c_void_p]
    L.mpo_profile.argtypes = [ctypes.c_void_p, c_double_p]
    L.nze_kernel_theta.argtypes = [ctypes.c_int32] * 4 + [
        ctypes.c_void_p, ctypes.c_void_p, c_double_p, ctypes.c_int32,
        ctypes.c_void_p, ctypes.c_void_p]
    L.nze_kernel_rowortho.argtypes = [
        ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
        c_double_p, c_int32_p, ctypes.c_void_p]
    L.nze_kernel_rowortho_static.argtypes = L.nze_kernel_rowortho.argtypes
    L.nze_server_create.argtypes = [ctypes.POINTER(ctypes.c_void_p),
                                    ctypes.c_void_p, ctypes.c_size_t,
                                    ctypes.c_int32, ctypes.c_void_p]
    L.nze_server_free.argtypes = [ctypes.c_void_p]
    L.nze_server_free.restype = None
    L.nze_server_submit.argtypes = [ctypes.c_void_p, ctypes.POINTER(NzeJobSpec),
                                    ctypes.POINTER(ctypes.c_int64)]
    L.nze_server_step.argtypes = [ctypes.c_void_p, c_int32_p, c_int32_p,
                                  c_int32_p]
    L.nze_server_poll.argtypes = [ctypes.c_void_p, ctypes.c_int64, c_int32_p,
                                  c_double_p, c_double_p, c_double_p]
    L.nze_server_stats.argtypes = [ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_size_t),
                                   ctypes.POINTER(ctypes.c_int64)]
    L.nze_fit_opts_default.argtypes = [ctypes.POINTER(NzeFitOpts)]
    L.nze_fit_opts_default.restype = None
    L.nze_extrapolate.argtypes = [ctypes.c_int32, c_double_p, c_double_p,
                                  c_double_p, ctypes.c_double, ctypes.c_int32,
                                  ctypes.POINTER(NzeFitOpts), c_double_p,
                                  c_double_p, c_uint8_p, c_int32_p]
    L.nze_fidelity_extrapolate.argtypes = [ctypes.c_int32, c_double_p,
                                           c_double_p, c_double_p, c_int32_p]
    L.nze_tune_footprint.argtypes = [ctypes.c_int32] * 3
    L.nze_tune_footprint.restype = ctypes.c_size_t
    L.nze_tune.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_void_p, ctypes.c_size_t,
                                                  ctypes.c_void_p, ctypes.POINTER(NzeTuning)]
    L.nze_tuning_get.argtypes = [ctypes.c_int32] * 3 + [ctypes.POINTER(NzeTuning)]
    L.nze_tuning_set.argtypes = [ctypes.c_int32] * 3 + [ctypes.POINTER(NzeTuning)]
    L.nze_shutdown.argtypes = []
    L.nze_shutdown.restype = None
    for fn in ("nze_strerror",):
        getattr(L, fn).argtypes = [ctypes.c_int]
        getattr(L, fn).restype = ctypes.c_char_p
    for fn in ("nze_last_error", "nze_version"):
        getattr(L, fn).argtypes = []
        getattr(L, fn).restype = ctypes.c_char_p
    _lib = L
    # release the library's staging buffers and events before the HIP
    # runtime is torn down at exit (atexit handlers run first)
    atexit.register(L.nze_shutdown)
    return L


def _check(rc):
    if rc != NZE_OK:
        raise NzeError(rc, lib().nze_last_error().decode())
    return rc


def _dp(a):
    return a.ctypes.data_as(c_double_p)


# ------------------------------------------------------------------ PTMs


def noise_struct(noise):
    """noise: dict with any of dep, ad, px, py, pz (or None)."""
    noise = noise or {}
    return NzeNoise(noise.get("dep", 0.0), noise.get("ad", 0.0),
                    noise.get("px", 0.0), noise.get("py", 0.0),
                    noise.get("pz", 0.0))


def build_ptm(U, noise=None, scale=1.0):
    U = np.asarray(U, dtype=np.complex128)
    re = np.ascontiguousarray(U.real)
    im = np.ascontiguousarray(U.imag)
    out = np.empty((16, 16))
    nz = noise_struct(noise)
    _check(lib().nze_build_ptm(_dp(re), _dp(im), ctypes.byref(nz),
                               float(scale), _dp(out)))
    return out


def build_ptm_pauli(U, rates, lam):
    """PTM of U followed by the two-qubit Pauli channel p_s = lam rates[s]."""
    U = np.asarray(U, dtype=np.complex128)
    re = np.ascontiguousarray(U.real)
    im = np.ascontiguousarray(U.imag)
    r = np.ascontiguousarray(rates, dtype=np.float64).reshape(16)
    out = np.empty((16, 16))
    _check(lib().nze_build_ptm_pauli(_dp(re), _dp(im), _dp(r), float(lam), _dp(out)))
    return out


def compose_1q(ptm16, u, rates, lam, qubit, after):
    """Folds the noisy single-qubit gate (u, then the Pauli channel
    p_s = lam rates[s]) on qubit 0/1 of the pair into ptm16, after or
    before it."""
    u = np.asarray(u, dtype=np.complex128)
    re = np.ascontiguousarray(u.real)
    im = np.ascontiguousarray(u.imag)
    r = np.ascontiguousarray(rates, dtype=np.float64).reshape(4)
    pin = np.ascontiguousarray(ptm16, dtype=np.float64)
    out = np.empty((16, 16))
    _check(lib().nze_ptm_compose_1q(_dp(pin), _dp(re), _dp(im), _dp(r), float(lam),
                                    int(qubit), int(bool(after)), _dp(out)))
    return out


def ptm_compose(first, second):
    """second @ first: the PTM of `first` followed by `second`."""
    a = np.ascontiguousarray(first, dtype=np.float64)
    b = np.ascontiguousarray(second, dtype=np.float64)
    out = np.empty((16, 16))
    _check(lib().nze_ptm_compose(_dp(a), _dp(b), _dp(out)))
    return out


def ptm_swap_qubits(ptm16):
    """The PTM with its two qubits exchanged (nze_ptm_swap_qubits)."""
    a = np.ascontiguousarray(ptm16, dtype=np.float64)
    out = np.empty((16, 16))
    _check(lib().nze_ptm_swap_qubits(_dp(a), _dp(out)))
    return out


SWAP_U = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]],
                  dtype=np.complex128)


def route_chain(n, pairs, restore=False):
    """nze_route_chain: ops [(site, gate index or -1 for a SWAP, flip)] of
    the gates on logical qubit pairs routed onto the chain (with the layout
    restored after every gate when ``restore``), and the final chain site of
    each logical qubit."""
    qa = np.ascontiguousarray([a for a, _ in pairs], dtype=np.int32)
    qb = np.ascontiguousarray([b for _, b in pairs], dtype=np.int32)
    cnt = ctypes.c_int32()
    perm = np.empty(n, dtype=np.int32)
    i32 = lambda a: a.ctypes.data_as(c_int32_p)
    _check(lib().nze_route_chain(n, len(pairs), i32(qa), i32(qb), int(bool(restore)), 0,
                                 None, None, None, ctypes.byref(cnt), None))
    k = cnt.value
    site = np.empty(k, dtype=np.int32)
    gate = np.empty(k, dtype=np.int32)
    flip = np.empty(k, dtype=np.uint8)
    _check(lib().nze_route_chain(n, len(pairs), i32(qa), i32(qb), int(bool(restore)), k,
                                 i32(site), i32(gate),
                                 flip.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                 ctypes.byref(cnt), i32(perm)))
    return list(zip(site.tolist(), gate.tolist(), flip.tolist())), perm


def routed_layers(n, gates, noise, factors, restore=False):
    """Gates (a, b, U) on logical qubit pairs as chain layers for
    MPO.apply_layer: the routed ops in order, consecutive ops on disjoint
    pairs grouped into one layer.  SWAPs are noiseless; a gate whose first
    qubit lands on the right of its pair takes the exchanged PTM.  Returns
    (layers as (left_sites, ptms[L][k][16][16]), final chain site of each
    logical qubit)."""
    ops, perm = route_chain(n, [(a, b) for a, b, _ in gates], restore)
    swap = build_ptm(SWAP_U)
    layers, cur, used = [], [], set()

    def flush():
        if cur:
            cur.sort(key=lambda o: o[0])
            ptms = np.empty((len(factors), len(cur), 16, 16))
            for j, c in enumerate(factors):
                for i, (s, g, f) in enumerate(cur):
                    if g < 0:
                        ptms[j, i] = swap
                    else:
                        r = build_ptm(gates[g][2], noise, c)
                        ptms[j, i] = ptm_swap_qubits(r) if f else r
            layers.append(([o[0] for o in cur], ptms))
        cur.clear()
        used.clear()

    for op in ops:
        if op[0] in used or op[0] + 1 in used:
            flush()
        cur.append(op)
        used.update((op[0], op[0] + 1))
    flush()
    return layers, perm


def permute_paulis(paulis, perm):
    """A Pauli string on logical qubits as the string on chain sites."""
    out = np.zeros(len(paulis), dtype=np.uint8)
    for q, p in enumerate(paulis):
        out[perm[q]] = p
    return out


def layer_ptms(unitaries, noise, factors):
    """[L][n_gates][16][16] PTMs of one layer at every level factor."""
    out = np.empty((len(factors), len(unitaries), 16, 16))
    for j, c in enumerate(factors):
        for i, U in enumerate(unitaries):
            out[j, i] = build_ptm(U, noise, c)
    return out


# ------------------------------------------------------------------ fits


def fit_opts(**kw):
    o = NzeFitOpts()
    lib().nze_fit_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def extrapolate(lam, values, fidelity=None, lam_target=0.0, method=NZE_POLY,
                **opts):
    """Returns (value, coef[3], used_mask, method_used)."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    val = np.ascontiguousarray(values, dtype=np.float64)
    fid = None if fidelity is None else np.ascontiguousarray(fidelity,
                                                             dtype=np.float64)
    out = ctypes.c_double()
    coef = np.zeros(3)
    used = np.zeros(lam.size, dtype=np.uint8)
    mu = ctypes.c_int32()
    o = fit_opts(**opts)
    _check(lib().nze_extrapolate(lam.size, _dp(lam), _dp(val),
                                 None if fid is None else _dp(fid),
                                 float(lam_target), method, ctypes.byref(o),
                                 ctypes.byref(out), _dp(coef),
                                 used.ctypes.data_as(c_uint8_p),
                                 ctypes.byref(mu)))
    return out.value, coef, used.astype(bool), mu.value


def fidelity_extrapolate(values, fids):
    v = np.ascontiguousarray(values, dtype=np.float64)
    f = np.ascontiguousarray(fids, dtype=np.float64)
    out = ctypes.c_double()
    conv = ctypes.c_int32()
    _check(lib().nze_fidelity_extrapolate(v.size, _dp(v), _dp(f),
                                          ctypes.byref(out),
                                          ctypes.byref(conv)))
    return out.value, bool(conv.value)


# ------------------------------------------------------ kernel-level hooks


def kernel_theta(A, B, ptm16, ltr=True):
    """Theta' of one two-site update from device tensors A ((4cl) x cm) and
    B (cm x (4cr)) in the path precision (torch float64 or float32)."""
    import torch
    prec = NZE_FP64 if A.dtype == torch.float64 else NZE_MIXED
    cl, cm = A.shape[0] // 4, A.shape[1]
    cr = B.shape[1] // 4
    X = torch.empty((4 * cl, 4 * cr) if ltr else (4 * cr, 4 * cl),
                    dtype=A.dtype, device=A.device)
    p = np.ascontiguousarray(ptm16, dtype=np.float64)
    _check(lib().nze_kernel_theta(prec, cl, cm, cr, A.data_ptr(), B.data_ptr(),
                                  _dp(p), int(ltr), X.data_ptr(),
                                  torch.cuda.current_stream().cuda_stream))
    return X


def kernel_rowortho(X, tol_rel, tol_abs, max_sweeps=40, W=None, static=False):
    """Block one-sided Jacobi on the rows of the device matrix X (in place);
    returns (W, squared row norms, sweeps).  static: the allocation-free entry
    point (nze_kernel_rowortho_static); W may then be passed in, so that the
    call allocates nothing."""
    import torch
    prec = NZE_FP64 if X.dtype == torch.float64 else NZE_MIXED
    R, C = X.shape
    if W is None:
        W = torch.empty((R, R), dtype=X.dtype, device=X.device)
    norms = np.zeros(R)
    sw = ctypes.c_int32()
    fn = lib().nze_kernel_rowortho_static if static else lib().nze_kernel_rowortho
    _check(fn(prec, R, C, X.data_ptr(), W.data_ptr(), tol_rel, tol_abs, max_sweeps,
              _dp(norms), ctypes.byref(sw), torch.cuda.current_stream().cuda_stream))
    return W, norms, sw.value


# ------------------------------------------------------------------ tuner

_TUNING_FIELDS = [f for f, _ in NzeTuning._fields_]


def tune(chi, precision, n_mpos, stream=None):
    """nze_tune: measures the candidate launch parameters for this batch
    shape on synthetic saturated blocks and caches the fastest; returns it."""
    import torch
    nbytes = int(lib().nze_tune_footprint(chi, precision, n_mpos))
    if nbytes == 0:
        raise NzeError(NZE_EINVAL, "invalid tuning shape")
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    ptr = (ws.data_ptr() + 255) & ~255
    st = stream if stream is not None else torch.cuda.current_stream()
    t = NzeTuning()
    _check(lib().nze_tune(chi, precision, n_mpos, ctypes.c_void_p(ptr),
                          ctypes.c_size_t(nbytes), ctypes.c_void_p(st.cuda_stream),
                          ctypes.byref(t)))
    del ws
    return {f: getattr(t, f) for f in _TUNING_FIELDS}


def tuning_get(chi, precision, n_mpos):
    """The cached tuning record for this shape, or None."""
    t = NzeTuning()
    if lib().nze_tuning_get(chi, precision, n_mpos, ctypes.byref(t)) != NZE_OK:
        return None
    return {f: getattr(t, f) for f in _TUNING_FIELDS}


def tuning_set(chi, precision, n_mpos, record):
    t = NzeTuning(*[record[f] for f in _TUNING_FIELDS])
    _check(lib().nze_tuning_set(chi, precision, n_mpos, ctypes.byref(t)))


# ------------------------------------------------------------------- MPOs


def make_config(n, chi, levels, precision=NZE_FP64, trunc_tol=0.0,
                tie_tol=0.0, jacobi_tol=0.0, jacobi_abs=0.0, max_sweeps=0,
                block=0):
    return MpoConfig(n, chi, levels, precision, trunc_tol, tie_tol,
                     jacobi_tol, jacobi_abs, max_sweeps, block)


def footprint(cfg):
    return int(lib().mpo_footprint(ctypes.byref(cfg)))


class MPO:
    """L vectorised MPOs (one per noise level) resident on the current GPU.

    The device workspace is a torch uint8 tensor owned by this object; the
    stream is torch's current stream unless one is given.
    """

    def __init__(self, n, chi, levels, precision=NZE_FP64, init_sites=None,
                 stream=None, **cfg_kw):
        import torch
        self.cfg = make_config(n, chi, levels, precision, **cfg_kw)
        nbytes = footprint(self.cfg)
        if nbytes == 0:
            raise NzeError(NZE_EINVAL, "invalid configuration")
        self.nbytes = nbytes
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self.ws.data_ptr()
        ptr = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.n, self.chi, self.levels = n, chi, levels
        h = ctypes.c_void_p()
        init = None
        if init_sites is not None:
            init = np.ascontiguousarray(init_sites, dtype=np.float64)
        _check(lib().mpo_init(ctypes.byref(h), ctypes.byref(self.cfg),
                              None if init is None else _dp(init),
                              ctypes.c_void_p(ptr), ctypes.c_size_t(nbytes),
                              ctypes.c_void_p(self.stream.cuda_stream)))
        self.h = h

    def apply_layer(self, left_sites, ptms):
        ls = np.ascontiguousarray(left_sites, dtype=np.int32)
        p = np.ascontiguousarray(ptms, dtype=np.float64)
        assert p.shape == (self.levels, ls.size, 16, 16)
        _check(lib().mpo_apply_layer(self.h, ls.size,
                                     ls.ctypes.data_as(c_int32_p), _dp(p)))

    def expect(self, observables, allow_nonfinite=False):
        """(values [L][n_obs], fidelity [L], trace [L]).  A level whose
        identity string was truncated away (trace 0) makes mpo_expect return
        NZE_ENUM; with allow_nonfinite the outputs are returned anyway."""
        obs = np.ascontiguousarray(np.asarray(observables, dtype=np.uint8)
                                   .reshape(-1, self.n))
        vals = np.zeros((self.levels, obs.shape[0]))
        fid = np.zeros(self.levels)
        tr = np.zeros(self.levels)
        rc = lib().mpo_expect(self.h, obs.shape[0],
                              obs.ctypes.data_as(c_uint8_p), _dp(vals),
                              _dp(fid), _dp(tr))
        if not (allow_nonfinite and rc == NZE_ENUM):
            _check(rc)
        return vals, fid, tr

    def stats(self):
        st = (NzeStats * self.levels)()
        bonds = np.zeros((self.levels, self.n - 1), dtype=np.int32)
        _check(lib().mpo_stats(self.h, st, bonds.ctypes.data_as(c_int32_p)))
        return [dict(fidelity=s.fidelity, log_scale=s.log_scale,
                     max_discarded=s.max_discarded,
                     min_cut_gap=s.min_cut_gap, max_bond=s.max_bond,
                     max_sweeps=s.max_sweeps, updates=s.updates,
                     sweeps_total=s.sweeps_total, flops=s.flops,
                     cap_hits=s.cap_hits, cap_offdiag=s.cap_offdiag,
                     ns_scaled=s.ns_scaled)
                for s in st], bonds

    def bond_spectrum(self, level, bond):
        """Schmidt values across bond (bond, bond + 1) of one level."""
        cap = 4 * self.chi
        out = np.zeros(cap)
        cnt = ctypes.c_int32()
        _check(lib().mpo_bond_spectrum(self.h, level, bond, _dp(out), cap,
                                       ctypes.byref(cnt)))
        return out[:min(cnt.value, cap)].copy()

    def entanglement_entropy(self, level, bond):
        """MPO entanglement entropy at bond (bond, bond + 1) of one level
        (mpo_bond_entropy)."""
        e = ctypes.c_double()
        _check(lib().mpo_bond_entropy(self.h, level, bond, ctypes.byref(e)))
        return e.value

    def true_fidelity(self, level, other, other_level):
        """F = |<<a|b>>|^2 / (||a||^2 ||b||^2) against level other_level of
        the MPO handle ``other`` (mpo_overlap)."""
        f, c = ctypes.c_double(), ctypes.c_double()
        _check(lib().mpo_overlap(self.h, level, other.h, other_level,
                                 ctypes.byref(f), ctypes.byref(c)))
        return f.value

    PROFILE_NAMES = ["theta", "gram", "check", "eigh", "rot_x", "rot_w",
                     "jacobi_wait", "norms", "select", "absorb", "move_prep",
                     "move_absorb", "sweep_overhead", "pair_solves", "wait_mean",
                     "jacobi_total"]

    def profile(self):
        out = np.zeros((self.levels, 16))
        _check(lib().mpo_profile(self.h, _dp(out)))
        return [dict(zip(self.PROFILE_NAMES, row)) for row in out]

    def sync(self):
        _check(lib().mpo_sync(self.h))

    def close(self):
        if self.h is not None and self.h.value:
            lib().mpo_free(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def apply_layer_batch(mpos, left_sites_list, ptms_list):
    """Advance several MPO handles by one layer each in shared launches."""
    k = len(mpos)
    hs = (ctypes.c_void_p * k)(*[m.h.value for m in mpos])
    ls_arrs = [np.ascontiguousarray(x, dtype=np.int32) for x in left_sites_list]
    p_arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in ptms_list]
    ng = np.array([a.size for a in ls_arrs], dtype=np.int32)
    lsp = (c_int32_p * k)(*[a.ctypes.data_as(c_int32_p) for a in ls_arrs])
    pp = (c_double_p * k)(*[_dp(a) for a in p_arrs])
    _check(lib().mpo_apply_layer_batch(hs, k, ng.ctypes.data_as(c_int32_p),
                                       lsp, pp))


def run_circuit(mpo, layers, noise, factors):
    """Apply every layer of ``layers`` (list of (left_sites, unitaries)) at all
    level factors."""
    for ls, us in layers:
        mpo.apply_layer(ls, layer_ptms(us, noise, factors))


# ---------------------------------------------------------------- serving


class Server:
    """Continuous-batching request loop of the library (nze_server_*): jobs
    are admitted by HBM footprint into a torch-allocated arena."""

    def __init__(self, arena_bytes, max_active=64, stream=None):
        import torch
        self.arena = torch.empty(arena_bytes + 256, dtype=torch.uint8,
                                 device="cuda")
        ptr = (self.arena.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(lib().nze_server_create(ctypes.byref(h), ctypes.c_void_p(ptr),
                                       ctypes.c_size_t(arena_bytes), max_active,
                                       ctypes.c_void_p(self.stream.cuda_stream)))
        self.h = h
        self.meta = {}

    def submit(self, n, chi, precision, layers, ptms, observables):
        """layers: list of left-site arrays; ptms: list of per-layer
        [L][gates][16][16] arrays (same length)."""
        L = ptms[0].shape[0] if ptms else 1
        gates = np.array([len(x) for x in layers], dtype=np.int32)
        ls = np.ascontiguousarray(np.concatenate(
            [np.asarray(x, dtype=np.int32) for x in layers]) if layers else
            np.zeros(0, dtype=np.int32))
        pt = np.ascontiguousarray(np.concatenate(
            [np.asarray(p, dtype=np.float64).reshape(-1) for p in ptms]) if ptms
            else np.zeros(0))
        obs = np.ascontiguousarray(np.asarray(observables, dtype=np.uint8)
                                   .reshape(-1, n))
        spec = NzeJobSpec(n, chi, L, precision, len(layers),
                          gates.ctypes.data_as(c_int32_p),
                          ls.ctypes.data_as(c_int32_p), _dp(pt), obs.shape[0],
                          obs.ctypes.data_as(c_uint8_p))
        jid = ctypes.c_int64()
        _check(lib().nze_server_submit(self.h, ctypes.byref(spec),
                                       ctypes.byref(jid)))
        self.meta[jid.value] = (L, obs.shape[0])
        return jid.value

    def step(self):
        a, q, d = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().nze_server_step(self.h, ctypes.byref(a), ctypes.byref(q),
                                     ctypes.byref(d)))
        return a.value, q.value, d.value

    def poll(self, jid):
        L, n_obs = self.meta[jid]
        st = ctypes.c_int32()
        vals = np.zeros((L, max(n_obs, 1)))
        fid = np.zeros(L)
        times = np.zeros(3)
        _check(lib().nze_server_poll(self.h, jid, ctypes.byref(st), _dp(vals),
                                     _dp(fid), _dp(times)))
        return st.value, vals[:, :n_obs], fid, times

    def stats(self):
        hw = ctypes.c_size_t()
        la = ctypes.c_int64()
        _check(lib().nze_server_stats(self.h, ctypes.byref(hw), ctypes.byref(la)))
        return hw.value, la.value

    def close(self):
        if self.h is not None and self.h.value:
            lib().nze_server_free(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
