"""ctypes marshalling for libelpahip.so (argument conversion only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libelpahip.so"

R64, R32, C64 = 0, 1, 2
PATH_AUTO, PATH_REF, PATH_STRIPE, PATH_SPLIT, PATH_WY = 0, 1, 2, 3, 4
ORDER_AUTO, ORDER_LINEAR, ORDER_XCD = 0, 1, 2
BATCH_AUTO, BATCH_ONE_LAUNCH, BATCH_DIAGONAL = 0, 1, 2

_lib = None


class ElpaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("elpa_hh error %d: %s" % (code, msg))
        self.code = code


class _Plan(C.Structure):
    _fields_ = [("path", C.c_int32), ("k", C.c_int32), ("steps", C.c_int32),
                ("order", C.c_int32), ("streams", C.c_int32), ("batch", C.c_int32)]


class _Problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("nev", C.c_int64), ("nbw", C.c_int64), ("ldq", C.c_int64),
                ("hh", C.c_void_p), ("tau", C.c_void_p), ("Q", C.c_void_p),
                ("dtype", C.c_int32), ("reserved", C.c_int32)]


class _Profile(C.Structure):
    _fields_ = [("kernel_ms", C.c_double), ("launches", C.c_int64), ("path", C.c_int32),
                ("k", C.c_int32), ("steps", C.c_int64), ("sum_launch_ms", C.c_double),
                ("streams", C.c_int32), ("reserved", C.c_int32)]


def library_path():
    return os.path.join(HERE, _LIB_NAME)


def library():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise ImportError("%s not built; run paper_1811_01277_amd/build.py" % path)
        L = C.CDLL(path)
        i64, i32, p = C.c_int64, C.c_int32, C.c_void_p
        L.elpa_hh_num_reflectors.argtypes = [i64, i64]
        L.elpa_hh_num_reflectors.restype = i64
        L.elpa_hh_slot_offset.argtypes = [i64, i64, i64]
        L.elpa_hh_slot_offset.restype = i64
        L.elpa_hh_trafo.argtypes = [i64, i64, i64, p, p, p, i64, i32, p]
        L.elpa_hh_trafo.restype = C.c_int
        L.elpa_hh_trafo_plan.argtypes = [i64, i64, i64, p, p, p, i64, i32, p, C.POINTER(_Plan)]
        L.elpa_hh_trafo_plan.restype = C.c_int
        L.elpa_hh_trafo_noalloc.argtypes = [i64, i64, i64, p, p, p, i64, i32, p]
        L.elpa_hh_trafo_noalloc.restype = C.c_int
        L.elpa_hh_batch_create.argtypes = [C.POINTER(_Problem), i64, C.POINTER(_Plan),
                                           C.POINTER(C.c_void_p)]
        L.elpa_hh_batch_create.restype = C.c_int
        L.elpa_hh_batch_run.argtypes = [p, p]
        L.elpa_hh_batch_run.restype = C.c_int
        L.elpa_hh_batch_bytes.argtypes = [p]
        L.elpa_hh_batch_bytes.restype = i64
        L.elpa_hh_batch_destroy.argtypes = [p]
        L.elpa_hh_batch_destroy.restype = C.c_int
        L.elpa_hh_trafo_batched.argtypes = [C.POINTER(_Problem), i64, p, C.POINTER(_Plan)]
        L.elpa_hh_trafo_batched.restype = C.c_int
        L.elpa_hh_chosen_plan.argtypes = [i64, i64, i64, i32, i32, C.POINTER(_Plan),
                                          C.POINTER(_Plan)]
        L.elpa_hh_chosen_plan.restype = C.c_int
        L.elpa_hh_plan_supported.argtypes = [i64, i32, C.POINTER(_Plan)]
        L.elpa_hh_plan_supported.restype = C.c_int
        L.elpa_hh_workspace_bytes.argtypes = [i64, i64, i64, i32, C.POINTER(_Plan)]
        L.elpa_hh_workspace_bytes.restype = i64
        L.elpa_hh_workspace_cached.argtypes = []
        L.elpa_hh_workspace_cached.restype = i64
        L.elpa_hh_workspace_release.argtypes = []
        L.elpa_hh_workspace_release.restype = i64
        L.elpa_hh_workspace_bytes_batched.argtypes = [C.POINTER(_Problem), i64,
                                                      C.POINTER(_Plan)]
        L.elpa_hh_workspace_bytes_batched.restype = i64
        L.elpa_hh_tune.argtypes = [i64, i64, i64, p, p, p, i64, i32, p, i32, C.POINTER(_Plan)]
        L.elpa_hh_tune.restype = C.c_int
        L.elpa_hh_autotune_setup.argtypes = [i32, i64, i64, i64, i32, C.POINTER(_Plan)]
        L.elpa_hh_autotune_setup.restype = p
        L.elpa_hh_autotune_step.argtypes = [p, p, p, p, i64, p, C.POINTER(i32)]
        L.elpa_hh_autotune_step.restype = C.c_int
        L.elpa_hh_autotune_best.argtypes = [p, C.POINTER(_Plan)]
        L.elpa_hh_autotune_best.restype = C.c_int
        L.elpa_hh_autotune_set_best.argtypes = [p]
        L.elpa_hh_autotune_set_best.restype = C.c_int
        L.elpa_hh_autotune_save.argtypes = [p, C.c_char_p]
        L.elpa_hh_autotune_save.restype = C.c_int
        L.elpa_hh_autotune_load.argtypes = [C.c_char_p]
        L.elpa_hh_autotune_load.restype = p
        L.elpa_hh_autotune_candidates.argtypes = [p]
        L.elpa_hh_autotune_candidates.restype = i64
        L.elpa_hh_autotune_free.argtypes = [p]
        L.elpa_hh_autotune_free.restype = None
        L.elpa_tridiag_eigh.argtypes = [i64, i64, p, p, p, p, i64, i32, p]
        L.elpa_tridiag_eigh.restype = C.c_int
        L.elpa_cholesky_inverse.argtypes = [i64, p, i64, i32, p, p]
        L.elpa_cholesky_inverse.restype = C.c_int
        L.elpa_generalized_to_standard.argtypes = [i64, p, i64, p, i64, i32, p]
        L.elpa_generalized_to_standard.restype = C.c_int
        L.elpa_generalized_back.argtypes = [i64, i64, p, i64, p, i64, i32, p]
        L.elpa_generalized_back.restype = C.c_int
        L.elpa_full_to_band.argtypes = [i64, i64, p, i64, p, i64, p, i32, p]
        L.elpa_full_to_band.restype = C.c_int
        L.elpa_band_to_tridiag.argtypes = [i64, i64, p, i64, p, p, p, p, i32, p]
        L.elpa_band_to_tridiag.restype = C.c_int
        L.elpa_bt2_trafo.argtypes = [i64, i64, i64, p, i64, p, p, i64, i32, p, i64]
        L.elpa_bt2_trafo.restype = C.c_int
        L.elpa_bt2_workspace_bytes.argtypes = [i64, i64, i64, i32, i64]
        L.elpa_bt2_workspace_bytes.restype = i64
        L.elpa_hh_tune_batched.argtypes = [C.POINTER(_Problem), i64, p, i32, C.POINTER(_Plan)]
        L.elpa_hh_tune_batched.restype = C.c_int
        L.elpa_hh_tuner_set.argtypes = [i32, i64, i64, i64, C.POINTER(_Plan)]
        L.elpa_hh_tuner_set.restype = C.c_int
        L.elpa_hh_tuner_get.argtypes = [i32, i64, i64, i64, C.POINTER(_Plan)]
        L.elpa_hh_tuner_get.restype = C.c_int
        L.elpa_hh_tuner_size.argtypes = []
        L.elpa_hh_tuner_size.restype = i64
        L.elpa_hh_tuner_clear.argtypes = []
        L.elpa_hh_tuner_clear.restype = None
        L.elpa_hh_tuner_save.argtypes = [C.c_char_p]
        L.elpa_hh_tuner_save.restype = C.c_int
        L.elpa_hh_tuner_load.argtypes = [C.c_char_p]
        L.elpa_hh_tuner_load.restype = C.c_int
        L.elpa_hh_profile_enable.argtypes = [C.c_int]
        L.elpa_hh_profile_enable.restype = C.c_int
        L.elpa_hh_profile_last.argtypes = [C.POINTER(_Profile)]
        L.elpa_hh_profile_last.restype = C.c_int
        L.elpa_strerror.argtypes = [C.c_int]
        L.elpa_strerror.restype = C.c_char_p
        L.elpa_hh_version.argtypes = []
        L.elpa_hh_version.restype = C.c_char_p
        _lib = L
    return _lib


def profile_enable(on=True):
    """Enable (or disable) kernel timing of the calls made from this thread."""
    rc = library().elpa_hh_profile_enable(1 if on else 0)
    if rc != 0:
        raise ElpaError(rc, strerror(rc))


def profile_last():
    """Timing of the latest call's main kernel sequence (waits for it):
    dict(kernel_ms, launches, path, k, steps, sum_launch_ms, streams)."""
    out = _Profile()
    rc = library().elpa_hh_profile_last(C.byref(out))
    if rc != 0:
        raise ElpaError(rc, strerror(rc))
    return {"kernel_ms": out.kernel_ms, "launches": out.launches, "path": out.path,
            "k": out.k, "steps": out.steps, "sum_launch_ms": out.sum_launch_ms,
            "streams": out.streams}


def _plan_dict(p):
    return {"path": p.path, "k": p.k, "steps": p.steps, "order": p.order, "streams": p.streams,
            "batch": p.batch}


def _check(rc):
    if rc != 0:
        raise ElpaError(rc, strerror(rc))


def tune(q, hh, tau, nbw, level=0, stream=None):
    """Time candidate plans for this problem (Q is not modified), cache the
    fastest for its size class and return it as a dict."""
    import torch
    n, nev = q.shape
    ldq = q.stride(1) if nev > 1 else max(n, 1)
    if stream is None:
        st = torch.cuda.current_stream(q.device).cuda_stream
    elif isinstance(stream, int):
        st = stream
    else:
        st = stream.cuda_stream
    out = _Plan()
    _check(library().elpa_hh_tune(n, nev, nbw, C.c_void_p(hh.data_ptr()),
                                  C.c_void_p(tau.data_ptr()), C.c_void_p(q.data_ptr()), ldq,
                                  _dtype_code(q), C.c_void_p(st), level, C.byref(out)))
    return _plan_dict(out)


def tuner_set(dtype, nbw, n, nev, path=0, k=0, steps=0, order=0, streams=0):
    pl = _Plan(path, k, steps, order, streams, 0)
    _check(library().elpa_hh_tuner_set(dtype, nbw, n, nev, C.byref(pl)))


def tuner_get(dtype, nbw, n, nev):
    """The cached plan of the size class of (n, nev) as a dict, or None."""
    out = _Plan()
    found = library().elpa_hh_tuner_get(dtype, nbw, n, nev, C.byref(out))
    return _plan_dict(out) if found == 1 else None


def tuner_size():
    return int(library().elpa_hh_tuner_size())


def tuner_clear():
    library().elpa_hh_tuner_clear()


def tuner_save(path):
    _check(library().elpa_hh_tuner_save(os.fsencode(path)))


def tuner_load(path):
    _check(library().elpa_hh_tuner_load(os.fsencode(path)))


def strerror(code):
    return library().elpa_strerror(code).decode()


def version():
    return library().elpa_hh_version().decode()


def num_reflectors(n, nbw):
    return int(library().elpa_hh_num_reflectors(n, nbw))


def slot_offset(n, nbw, s):
    return int(library().elpa_hh_slot_offset(n, nbw, s))


def _plan(path, k, steps=0, order=0, streams=0, batch=0):
    if path is None and not k and not steps and not order and not streams and not batch:
        return None
    return _Plan(int(path or 0), int(k or 0), int(steps or 0), int(order or 0),
                 int(streams or 0), int(batch or 0))


def plan_supported(nbw, dtype, path=PATH_AUTO, k=0):
    pl = _plan(path, k)
    return bool(library().elpa_hh_plan_supported(nbw, dtype, C.byref(pl) if pl else None))


def chosen_plan(n, nev, nbw, dtype, batched=False, path=None, k=0):
    """The plan (path, k filled in) a single or batched call runs for this
    problem size (elpa_hh_chosen_plan)."""
    pl = _plan(path, k)
    out = _Plan()
    _check(library().elpa_hh_chosen_plan(n, nev, nbw, dtype, 1 if batched else 0,
                                         C.byref(pl) if pl is not None else None,
                                         C.byref(out)))
    return _plan_dict(out)


def workspace_bytes(n, nev, nbw, dtype, path=None, k=0):
    """Device bytes one call allocates for this problem and plan (-1: invalid)."""
    pl = _plan(path, k)
    return int(library().elpa_hh_workspace_bytes(n, nev, nbw, dtype,
                                                 C.byref(pl) if pl is not None else None))


def workspace_cached():
    """Device bytes the library's workspace cache holds on the current device."""
    return int(library().elpa_hh_workspace_cached())


def workspace_release():
    """Free the cache's idle workspace blocks on the current device (returns
    the bytes freed)."""
    return int(library().elpa_hh_workspace_release())


def workspace_bytes_batched(problems, path=None, k=0):
    """Upper bound of the device bytes hh_trafo_batched allocates for a list
    of (n, nev, nbw, dtype code) tuples (-1: invalid)."""
    arr = (_Problem * max(1, len(problems)))()
    for i, (n, nev, nbw, dt) in enumerate(problems):
        arr[i] = _Problem(n, nev, nbw, max(n, 1), None, None, None, dt, 0)
    pl = _plan(path, k)
    return int(library().elpa_hh_workspace_bytes_batched(
        arr, len(problems), C.byref(pl) if pl is not None else None))


def hh_trafo_ptr(n, nev, nbw, hh, tau, q, ldq, dtype, stream=0, path=None, k=0, steps=0,
                 order=0, streams=0):
    """Raw-pointer entry: returns the library's status code (no raise)."""
    pl = _plan(path, k, steps, order, streams)
    return int(library().elpa_hh_trafo_plan(
        n, nev, nbw, C.c_void_p(hh), C.c_void_p(tau), C.c_void_p(q), ldq, dtype,
        C.c_void_p(stream), C.byref(pl) if pl is not None else None))


# fixed device scratch of the allocation-free entry point (include/elpa_hh.h)
NOALLOC_SCRATCH_BYTES = 256 << 20


def hh_trafo_noalloc_ptr(n, nev, nbw, hh, tau, q, ldq, dtype, stream=0):
    """Raw-pointer allocation-free entry (elpa_hh_trafo_noalloc): returns the
    library's status code (no raise)."""
    return int(library().elpa_hh_trafo_noalloc(
        n, nev, nbw, C.c_void_p(hh), C.c_void_p(tau), C.c_void_p(q), ldq, dtype,
        C.c_void_p(stream)))


def _dtype_code(t):
    import torch
    m = {torch.float64: R64, torch.float32: R32, torch.complex128: C64}
    if t.dtype not in m:
        raise TypeError("unsupported dtype %s" % t.dtype)
    return m[t.dtype]


def hh_trafo(q, hh, tau, nbw, stream=None, path=None, k=0, steps=0, order=0, streams=0,
             batch=0):
    """Q <- H(0,0) ... H(n-2,J-1) Q in place on a column-major torch tensor.

    q:   (n, nev) device tensor with q.stride(0) == 1 (column major, ldq =
         q.stride(1)); float64, float32 or complex128.
    hh:  1-D contiguous tensor of N_refl*nbw reflector entries (same dtype).
    tau: 1-D contiguous tensor of N_refl scalars (same dtype).
    stream: torch.cuda.Stream or raw hipStream_t int; default: current stream.
    path, k, steps, order, streams: explicit plan (elpa_hh_plan); 0 / None =
    library choice.  batch: the batched-schedule field of a plan (accepted so
    that a tuned plan dict can be passed; a single call ignores it).
    """
    import torch
    if q.dim() != 2:
        raise ValueError("q must be 2-D (n, nev)")
    n, nev = q.shape
    if n > 1 and nev > 0 and q.stride(0) != 1:
        raise ValueError("q must be column major (stride(0) == 1)")
    ldq = q.stride(1) if nev > 1 else max(n, 1)
    dt = _dtype_code(q)
    if hh.dtype != q.dtype or tau.dtype != q.dtype:
        raise TypeError("hh, tau and q must share a dtype")
    if not (hh.is_contiguous() and tau.is_contiguous()):
        raise ValueError("hh and tau must be contiguous")
    nr = num_reflectors(n, nbw) if n > 1 else 0
    if nr > 0 and (hh.numel() < nr * nbw or tau.numel() < nr):
        raise ValueError("hh needs %d and tau %d elements" % (nr * nbw, nr))
    for t in (q, hh, tau):
        if n > 1 and nev > 0 and not t.is_cuda:
            raise ValueError("q, hh and tau must be device tensors")
    if stream is None:
        st = torch.cuda.current_stream(q.device).cuda_stream if q.is_cuda else 0
    elif isinstance(stream, int):
        st = stream
    else:
        st = stream.cuda_stream
    rc = hh_trafo_ptr(n, nev, nbw, hh.data_ptr(), tau.data_ptr(), q.data_ptr(), ldq, dt, st,
                      path, k, steps, order, streams)
    if rc != 0:
        raise ElpaError(rc, strerror(rc))
    return q


def _marshal_batch(problems, stream):
    """C problem array and raw stream of a list of (q, hh, tau, nbw) tuples."""
    import torch
    arr = (_Problem * max(1, len(problems)))()
    dev = None
    for i, (q, hh, tau, nbw) in enumerate(problems):
        n, nev = q.shape
        if n > 1 and nev > 0 and q.stride(0) != 1:
            raise ValueError("q must be column major (stride(0) == 1)")
        if hh.dtype != q.dtype or tau.dtype != q.dtype:
            raise TypeError("hh, tau and q must share a dtype")
        nr = num_reflectors(n, nbw) if n > 1 else 0
        if nr > 0 and (hh.numel() < nr * nbw or tau.numel() < nr):
            raise ValueError("problem %d: hh needs %d and tau %d elements" % (i, nr * nbw, nr))
        ldq = q.stride(1) if nev > 1 else max(n, 1)
        arr[i] = _Problem(n, nev, nbw, ldq, hh.data_ptr(), tau.data_ptr(), q.data_ptr(),
                          _dtype_code(q), 0)
        dev = q.device if dev is None else dev
    if stream is None:
        st = torch.cuda.current_stream(dev).cuda_stream if dev is not None and dev.type == "cuda" else 0
    elif isinstance(stream, int):
        st = stream
    else:
        st = stream.cuda_stream
    return arr, st


def hh_trafo_batched_ptr(problems, stream=0, path=None, k=0, steps=0, order=0, streams=0,
                         batch=0):
    """Raw-pointer batched entry over (n, nev, nbw, ldq, hh, tau, q, dtype code)
    tuples: returns the library's status code (no raise)."""
    arr = (_Problem * max(1, len(problems)))()
    for i, (n, nev, nbw, ldq, hh, tau, q, dt) in enumerate(problems):
        arr[i] = _Problem(n, nev, nbw, ldq, hh, tau, q, dt, 0)
    pl = _plan(path, k, steps, order, streams, batch)
    return int(library().elpa_hh_trafo_batched(arr, len(problems), C.c_void_p(stream),
                                                C.byref(pl) if pl is not None else None))


def hh_trafo_batched(problems, stream=None, path=None, k=0, steps=0, order=0, streams=0,
                     batch=0):
    """Batched Q <- H ... H Q over a list of (q, hh, tau, nbw) tensor tuples.

    Each q is a column-major (n, nev) device tensor as in hh_trafo; problems
    may differ in n, nev and dtype.  The problems of one (dtype, nbw) group
    that run the two-lane kernel are back-transformed in one kernel launch
    (one workgroup per 32-column stripe of a problem, largest problems first);
    groups run in order on one stream.  batch: BATCH_ONE_LAUNCH or
    BATCH_DIAGONAL forces that schedule of the two-lane kernel (default: the
    library's model picks).
    """
    arr, st = _marshal_batch(problems, stream)
    pl = _plan(path, k, steps, order, streams, batch)
    rc = int(library().elpa_hh_trafo_batched(arr, len(problems), C.c_void_p(st),
                                              C.byref(pl) if pl is not None else None))
    if rc != 0:
        raise ElpaError(rc, strerror(rc))
    return problems


class Batch:
    """A prepared batched call (elpa_hh_batch_*): the schedule, workspace and
    descriptor tables of a list of (q, hh, tau, nbw) problems are set up once;
    run() then only launches kernels, so it can be captured into a CUDA/HIP
    graph (torch.cuda.graph) and replayed.  The tensors must stay alive (and
    in place) as long as the Batch.  Runs of one Batch must not overlap."""

    def __init__(self, problems, path=None, k=0, steps=0, order=0, streams=0, batch=0):
        arr, _ = _marshal_batch(problems, 0)
        pl = _plan(path, k, steps, order, streams, batch)
        h = C.c_void_p()
        _check(library().elpa_hh_batch_create(arr, len(problems),
                                               C.byref(pl) if pl is not None else None,
                                               C.byref(h)))
        self._h = h
        self._keep = list(problems)      # the device buffers the batch points to

    @property
    def nbytes(self):
        return int(library().elpa_hh_batch_bytes(self._h))

    def run(self, stream=None):
        import torch
        if stream is None:
            st = torch.cuda.current_stream().cuda_stream
        elif isinstance(stream, int):
            st = stream
        else:
            st = stream.cuda_stream
        _check(library().elpa_hh_batch_run(self._h, C.c_void_p(st)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            library().elpa_hh_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_batched(problems, level=0, stream=None):
    """Time uniform plans over the whole batch (the Q tensors are not
    modified) and return the fastest as a dict, to pass to hh_trafo_batched
    as keyword arguments.  Not cached."""
    arr, st = _marshal_batch(problems, stream)
    out = _Plan()
    _check(library().elpa_hh_tune_batched(arr, len(problems), C.c_void_p(st), level,
                                           C.byref(out)))
    return _plan_dict(out)


def bt2_trafo(q, v, tau, nbw, stream=None, block=0):
    """Band -> full back-transformation Q <- H_0 ... H_{n-nbw-1} Q in place
    (include/elpa_bt2.h).

    q:   (n, nev) column-major device tensor (float64, float32, complex128).
    v:   column-major device tensor with n rows (leading dimension
         v.stride(1) >= n) and at least n - nbw columns; column c holds v_c on
         rows c+nbw+1 .. n-1 (its unit lead at row c+nbw and everything above
         are not read).
    tau: 1-D contiguous tensor of at least n - nbw scalars (same dtype).
    block: reflectors per compact-WY block (0 = library choice).
    """
    import torch
    if q.dim() != 2 or v.dim() != 2:
        raise ValueError("q and v must be 2-D")
    n, nev = q.shape
    if n > 1 and nev > 0 and q.stride(0) != 1:
        raise ValueError("q must be column major (stride(0) == 1)")
    if v.shape[0] != n or (v.shape[1] > 1 and v.stride(0) != 1):
        raise ValueError("v must be column major with n rows")
    nref = max(0, n - nbw)
    if v.shape[1] < nref or tau.numel() < nref:
        raise ValueError("v needs %d columns and tau %d elements" % (nref, nref))
    if v.dtype != q.dtype or tau.dtype != q.dtype:
        raise TypeError("q, v and tau must share a dtype")
    if not tau.is_contiguous():
        raise ValueError("tau must be contiguous")
    ldq = q.stride(1) if nev > 1 else max(n, 1)
    ldv = v.stride(1) if v.shape[1] > 1 else max(n, 1)
    if stream is None:
        st = torch.cuda.current_stream(q.device).cuda_stream if q.is_cuda else 0
    elif isinstance(stream, int):
        st = stream
    else:
        st = stream.cuda_stream
    rc = int(library().elpa_bt2_trafo(n, nev, nbw, C.c_void_p(v.data_ptr()), ldv,
                                      C.c_void_p(tau.data_ptr()), C.c_void_p(q.data_ptr()), ldq,
                                      _dtype_code(q), C.c_void_p(st), int(block)))
    if rc != 0:
        raise ElpaError(rc, strerror(rc))
    return q


def bt2_workspace_bytes(n, nev, nbw, dtype, block=0):
    """Device bytes one bt2_trafo call allocates (-1: invalid)."""
    return int(library().elpa_bt2_workspace_bytes(n, nev, nbw, dtype, block))


def band_to_tridiag(a, nbw, stream=None):
    """Band -> tridiagonal reduction on the device (include/elpa_b2t.h).

    a: (n, n) column-major device tensor (float64 or complex128), a Hermitian
       band matrix of semi-bandwidth nbw in full storage; overwritten.
    Returns (d, e, hh, tau): float64 device tensors of the diagonal (n) and
    subdiagonal (n-1), and the reflectors in hh_trafo's layout (tensors of
    a's dtype), all produced on the device.
    """
    import torch
    if a.dim() != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("a must be square")
    n = a.shape[0]
    if n > 1 and a.stride(0) != 1:
        raise ValueError("a must be column major (stride(0) == 1)")
    lda = a.stride(1) if n > 1 else 1
    nr = num_reflectors(n, nbw) if n > 1 else 0
    dev = a.device
    d = torch.empty(n, dtype=torch.float64, device=dev)
    e = torch.empty(max(n - 1, 1), dtype=torch.float64, device=dev)
    hh = torch.empty(max(nr * nbw, 1), dtype=a.dtype, device=dev)
    tau = torch.empty(max(nr, 1), dtype=a.dtype, device=dev)
    if stream is None:
        st = torch.cuda.current_stream(dev).cuda_stream if a.is_cuda else 0
    elif isinstance(stream, int):
        st = stream
    else:
        st = stream.cuda_stream
    rc = int(library().elpa_band_to_tridiag(n, nbw, C.c_void_p(a.data_ptr()), lda,
                                            C.c_void_p(d.data_ptr()), C.c_void_p(e.data_ptr()),
                                            C.c_void_p(hh.data_ptr()),
                                            C.c_void_p(tau.data_ptr()), _dtype_code(a),
                                            C.c_void_p(st)))
    if rc != 0:
        raise ElpaError(rc, strerror(rc))
    return d, e[:max(n - 1, 0)], hh[:nr * nbw], tau[:nr]


AUTOTUNE_FAST, AUTOTUNE_MEDIUM = 0, 1


class Autotune:
    """On-the-fly autotuning over a sequence of similar solves
    (elpa_hh_autotune_* in include/elpa_hh.h): every step() is one real
    back-transformation with the next candidate setting; once all have been
    timed, steps run the fastest.

        at = Autotune(AUTOTUNE_MEDIUM, n, nev, nbw, R64)
        for each SCF step:  tuning = at.step(q, hh, tau)
        at.set_best()   # plain hh_trafo calls of this size class use it
    """

    def __init__(self, level, n, nev, nbw, dtype, path=0, k=0, steps=0, streams=0, _state=None):
        if _state is not None:
            self._st = _state
        else:
            fixed = _plan(path or None, k, steps, 0, streams)
            self._st = library().elpa_hh_autotune_setup(
                level, n, nev, nbw, dtype, C.byref(fixed) if fixed is not None else None)
            if not self._st:
                raise ElpaError(-1, "autotune setup refused (arguments or no candidate)")

    @classmethod
    def load(cls, path):
        st = library().elpa_hh_autotune_load(os.fsencode(path))
        if not st:
            raise ElpaError(-1, "autotune state file does not parse")
        return cls(0, 0, 0, 0, 0, _state=st)

    @property
    def candidates(self):
        return int(library().elpa_hh_autotune_candidates(self._st))

    def step(self, q, hh, tau, stream=None):
        """One solve (Q <- H ... H Q in place); returns True while tuning."""
        import torch
        n, nev = q.shape
        ldq = q.stride(1) if nev > 1 else max(n, 1)
        if stream is None:
            st = torch.cuda.current_stream(q.device).cuda_stream
        elif isinstance(stream, int):
            st = stream
        else:
            st = stream.cuda_stream
        tuning = C.c_int32(0)
        _check(library().elpa_hh_autotune_step(
            self._st, C.c_void_p(hh.data_ptr()), C.c_void_p(tau.data_ptr()),
            C.c_void_p(q.data_ptr()), ldq, C.c_void_p(st), C.byref(tuning)))
        return bool(tuning.value)

    def best(self):
        out = _Plan()
        _check(library().elpa_hh_autotune_best(self._st, C.byref(out)))
        return _plan_dict(out)

    def set_best(self):
        _check(library().elpa_hh_autotune_set_best(self._st))

    def save(self, path):
        _check(library().elpa_hh_autotune_save(self._st, os.fsencode(path)))

    def close(self):
        if getattr(self, "_st", None):
            library().elpa_hh_autotune_free(self._st)
            self._st = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def full_to_band(a, nbw, stream=None):
    """Full -> band reduction on the device (include/elpa_f2b.h).

    a: (n, n) column-major device tensor (float64 or complex128), a Hermitian
       matrix in full storage; overwritten with the band matrix (the input of
       band_to_tridiag).
    Returns (v, tau): the reflectors in bt2_trafo's layout, device tensors of
    a's dtype (v column major, n x max(n-nbw, 1)).
    """
    import torch
    if a.dim() != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("a must be square")
    n = a.shape[0]
    if n > 1 and a.stride(0) != 1:
        raise ValueError("a must be column major (stride(0) == 1)")
    lda = a.stride(1) if n > 1 else 1
    N = max(n - nbw, 1)
    v = torch.zeros((N, n), dtype=a.dtype, device=a.device).t()
    tau = torch.zeros(N, dtype=a.dtype, device=a.device)
    if stream is None:
        st = torch.cuda.current_stream(a.device).cuda_stream if a.is_cuda else 0
    elif isinstance(stream, int):
        st = stream
    else:
        st = stream.cuda_stream
    rc = int(library().elpa_full_to_band(n, nbw, C.c_void_p(a.data_ptr()), lda,
                                         C.c_void_p(v.data_ptr()), max(n, 1),
                                         C.c_void_p(tau.data_ptr()), _dtype_code(a),
                                         C.c_void_p(st)))
    if rc != 0:
        raise ElpaError(rc, strerror(rc))
    return v, tau


def _stream_of(t, stream):
    import torch
    if stream is None:
        return torch.cuda.current_stream(t.device).cuda_stream if t.is_cuda else 0
    return stream if isinstance(stream, int) else stream.cuda_stream


def _col_major_ld(x, name):
    if x.dim() != 2:
        raise ValueError(f"{name} must be a matrix")
    if x.shape[0] > 1 and x.stride(0) != 1:
        raise ValueError(f"{name} must be column major (stride(0) == 1)")
    return max(x.stride(1) if x.shape[1] > 1 else x.shape[0], 1)


def cholesky_inverse(b, stream=None, check=True):
    """b <- L^{-1} with b = L L^H (include/elpa_gen.h): the inverted Cholesky
    factor that the generalized solve keeps in b's storage.  b: (n, n)
    column-major device tensor (float64 or complex128), lower triangle read.
    With check=True the stream is synchronised and a matrix that is not
    positive definite raises numpy.linalg.LinAlgError; with check=False the
    device int32 info tensor is returned (0, or the 1-based order of the
    first leading minor that is not positive definite)."""
    import torch
    if b.dim() != 2 or b.shape[0] != b.shape[1]:
        raise ValueError("b must be square")
    n = b.shape[0]
    ldb = _col_major_ld(b, "b")
    info = torch.zeros(1, dtype=torch.int32, device=b.device)
    rc = int(library().elpa_cholesky_inverse(n, C.c_void_p(b.data_ptr()), ldb, _dtype_code(b),
                                             C.c_void_p(_stream_of(b, stream)),
                                             C.c_void_p(info.data_ptr())))
    if rc != 0:
        raise ElpaError(rc, strerror(rc))
    if not check:
        return info
    i = int(info.item())
    if i:
        import numpy as np
        raise np.linalg.LinAlgError(f"leading minor of order {i} is not positive definite")
    return info


def generalized_to_standard(a, linv, stream=None):
    """a <- linv a linv^H, exactly Hermitian (include/elpa_gen.h)."""
    if a.dim() != 2 or a.shape[0] != a.shape[1] or tuple(linv.shape) != tuple(a.shape):
        raise ValueError("a and linv must be square of the same size")
    if linv.dtype != a.dtype:
        raise ValueError("a and linv must have the same dtype")
    rc = int(library().elpa_generalized_to_standard(
        a.shape[0], C.c_void_p(a.data_ptr()), _col_major_ld(a, "a"), C.c_void_p(linv.data_ptr()),
        _col_major_ld(linv, "linv"), _dtype_code(a), C.c_void_p(_stream_of(a, stream))))
    if rc != 0:
        raise ElpaError(rc, strerror(rc))


def generalized_back(q, linv, stream=None):
    """q <- linv^H q: the generalized problem's eigenvectors from the standard
    problem's (include/elpa_gen.h)."""
    if q.dim() != 2 or linv.dim() != 2 or linv.shape[0] != linv.shape[1] \
            or linv.shape[0] != q.shape[0]:
        raise ValueError("q must have as many rows as the square linv")
    if linv.dtype != q.dtype:
        raise ValueError("q and linv must have the same dtype")
    rc = int(library().elpa_generalized_back(
        q.shape[0], q.shape[1], C.c_void_p(linv.data_ptr()), _col_major_ld(linv, "linv"),
        C.c_void_p(q.data_ptr()), _col_major_ld(q, "q"), _dtype_code(q),
        C.c_void_p(_stream_of(q, stream))))
    if rc != 0:
        raise ElpaError(rc, strerror(rc))


def tridiag_eigh(d, e, nev=None, dtype=None, stream=None):
    """Eigenvalues and eigenvectors of the symmetric tridiagonal matrix
    (d, e) by divide and conquer on the device (include/elpa_tridiag.h).

    d: (n,) float64 device tensor, e: (n-1,) float64 device tensor.
    Returns (lam, z): all n eigenvalues ascending, and the eigenvectors of the
    nev (default n) smallest as an (n, nev) column-major tensor of dtype
    (float64 default; float32 or complex128 to feed hh_trafo directly)."""
    import torch
    n = d.shape[0]
    nev = n if nev is None else int(nev)
    dtype = torch.float64 if dtype is None else dtype
    if d.dtype != torch.float64 or e.dtype != torch.float64:
        raise TypeError("d and e must be float64")
    if e.shape[0] != max(n - 1, 0):
        raise ValueError("e must have n - 1 entries")
    d = d.contiguous()
    e = e.contiguous()
    lam = torch.empty(n, dtype=torch.float64, device=d.device)
    z = torch.empty((max(nev, 1), max(n, 1)), dtype=dtype, device=d.device).t()[:n, :nev]
    rc = int(library().elpa_tridiag_eigh(
        n, nev, C.c_void_p(d.data_ptr()), C.c_void_p(e.data_ptr() if n > 1 else 0),
        C.c_void_p(lam.data_ptr()), C.c_void_p(z.data_ptr() if nev > 0 else 0), max(n, 1),
        _dtype_code(z), C.c_void_p(_stream_of(d, stream))))
    if rc != 0:
        raise ElpaError(rc, strerror(rc))
    return lam, z


def eigenvectors(a, nev=None, nbw=64, stream=None):
    """The whole standard eigensolver on the device, the C-ABI stages in
    order: full -> band (elpa_full_to_band), band -> tridiagonal
    (elpa_band_to_tridiag), divide and conquer (elpa_tridiag_eigh),
    tridiagonal -> band (elpa_hh_trafo) and band -> full (elpa_bt2_trafo).

    a: (n, n) column-major device tensor, float64 or complex128, Hermitian in
       full storage; overwritten (it holds the band matrix afterwards).
    Returns (lam, z): all n eigenvalues ascending (float64) and the
    eigenvectors of the nev (default n) smallest as an (n, nev) column-major
    tensor of a's dtype."""
    n = a.shape[0]
    nev = n if nev is None else int(nev)
    if n <= 1:
        import torch
        lam = a.diagonal().real.to(torch.float64).clone() if n else \
            torch.empty(0, dtype=torch.float64, device=a.device)
        z = torch.ones((n, nev), dtype=a.dtype, device=a.device)
        return lam, z
    b = max(1, min(nbw, n - 1))
    v, t1 = full_to_band(a, b, stream)
    d, e, hh, tau = band_to_tridiag(a, b, stream)
    lam, z = tridiag_eigh(d, e, nev, a.dtype, stream)
    if nev > 0:
        hh_trafo(z, hh, tau, b, stream)
        bt2_trafo(z, v, t1, b, stream=stream)
    return lam, z


def generalized_eigenvectors(a, b, nev=None, nbw=64, is_already_decomposed=False,
                             stream=None):
    """A V = B V Lambda on the device (Hermitian A, Hermitian positive
    definite B).  Unless is_already_decomposed, b is overwritten by the
    inverse of its Cholesky factor (cholesky_inverse); a later call with the
    same B passes that b with is_already_decomposed=True and skips the
    factorisation.  a is overwritten.  Returns (lam, v) as eigenvectors()."""
    if not is_already_decomposed:
        cholesky_inverse(b, stream)
    generalized_to_standard(a, b, stream)
    lam, z = eigenvectors(a, nev, nbw, stream)
    if z.shape[1] > 0:
        generalized_back(z, b, stream)
    return lam, z
