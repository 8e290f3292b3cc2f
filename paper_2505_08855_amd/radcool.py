"""ctypes binding of libradcool.so (include/radcool.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Device buffers are torch tensors on the current HIP device (torch is
used for allocation and streams, nothing else).  A missing or unbuilt library
raises ``RadcoolError``; there is no fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libradcool.so")

RC_OK = 0
STATUS_NAMES = {-1: "RC_EINVAL", -2: "RC_ENOMEM", -3: "RC_EDEVICE", -4: "RC_EUNSUPPORTED",
                -5: "RC_ESTATE", -6: "RC_EIO"}

TAB_BREM, TAB_SYNCH, TAB_ETA, TAB_COUL = 0, 1, 2, 3
ST_INVALID, ST_CLAMP_COOL, ST_CLAMP_COUL, ST_FLOOR, ST_MAXITER, ST_GAS_FLOOR, ST_NO_RATE = 1, 2, 4, 8, 16, 32, 64
SCHEME_NEWTON, SCHEME_EXPLICIT16, SCHEME_RATES = 0, 1, 2
VARIANT_AUTO, VARIANT_GLOBAL, VARIANT_LDS, VARIANT_TEX, VARIANT_DIRECT = 0, 1, 2, 3, 4
VARIANTS = {"auto": 0, "global": 1, "lds": 2, "tex": 3, "direct": 4, "cell": 5}
SCHEMES = {"newton": 0, "explicit16": 1, "rates": 2}

EXPORTED = ("rc_default_spec", "rc_default_opts", "rc_build_tables", "rc_tables_import",
            "rc_tables_export", "rc_tables_info", "rc_tables_save", "rc_tables_load", "rc_tables_storage_bytes",
            "rc_tables_destroy", "rc_cool_step", "rc_cool_step_noalloc", "rc_constants", "rc_selftest_node_host",
            "rc_selftest_special_host", "rc_selftest_step_host", "rc_last_error",
            "rc_cool_step_backward", "rc_selftest_backward_host", "rc_cool_step_batched",
            "rc_plan_create", "rc_plan_launch", "rc_plan_info", "rc_plan_destroy",
            "rc_disk_inputs", "rc_rad_pressure_correction", "rc_selftest_disk_host", "rc_selftest_radp_host",
            "rc_paper_axes4", "rc_build_table4d", "rc_table4d_import", "rc_table4d_export", "rc_table4d_destroy",
            "rc_rates4d", "rc_selftest_node4d_host", "rc_selftest_rates4d_host", "rc_apply_cooling",
            "rc_selftest_coupling_host", "rc_batched_workgroup_items", "rc_plan_workgroup_items")
MAX_STATES = 64
NOALLOC_MAX_CELLS = 1 << 20      # RC_NOALLOC_MAX_CELLS


class RadcoolError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, str(code)), msg))
        self.code = code


class Axes(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]


VALUE_DTYPES = {"f32": 0, "bf16": 1}
COMPTON = {"derived": 0, "literal": 1}
THETA_I_MASS = {"m_p": 0, "m_e": 1}
RATE_DTYPES = {"f64": 0, "f32": 1}


class TableSpec(ctypes.Structure):
    _fields_ = [("cool", Axes), ("coul", Axes), ("ln_lambda", ctypes.c_double),
                ("value_dtype", ctypes.c_int32), ("compton_exponent", ctypes.c_int32),
                ("theta_i_mass", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("external_storage", ctypes.c_void_p), ("external_bytes", ctypes.c_uint64)]


class State(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in ("n_e", "T_e", "T_i", "B", "H", "T_floor_gas")]


def _state(state):
    """rc_state from a dict of device tensors (T_floor_gas optional)."""
    fl = state.get("T_floor_gas")
    return State(*[state[k].data_ptr() for k in ("n_e", "T_e", "T_i", "B", "H")],
                 fl.data_ptr() if fl is not None else None)


class Out(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in ("T_e_new", "T_i_new", "Q_rad", "Q_cc", "status",
                                               "Q_brem", "Q_syn", "eta")]


class Fwd(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in ("T_e_new", "T_i_new", "status")]


class Cotangent(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in ("T_e_new", "T_i_new", "Q_rad", "Q_cc")]


class Grad(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in ("n_e", "T_e", "T_i", "B", "H", "tables")]


class DiskParams(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("spin", ctypes.c_double), ("h_floor", ctypes.c_double),
                ("r_g", ctypes.c_double)]


class Coupling(ctypes.Structure):
    _fields_ = [("u_cov", ctypes.c_void_p * 4), ("sqrt_g", ctypes.c_void_p), ("U", ctypes.c_void_p * 4)]


class Axes4(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 4), ("lo", ctypes.c_double * 4), ("hi", ctypes.c_double * 4)]


class Block(ctypes.Structure):
    _fields_ = [("first_cell", ctypes.c_int64), ("n_cells", ctypes.c_int32), ("state_id", ctypes.c_int32)]


BLOCK_DTYPE = np.dtype([("first_cell", np.int64), ("n_cells", np.int32), ("state_id", np.int32)])


class StepOpts(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int32), ("variant", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("block", ctypes.c_int32), ("T_floor", ctypes.c_double), ("tol", ctypes.c_double),
                ("passes", ctypes.c_int32), ("grid", ctypes.c_int32), ("rate_dtype", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None


def lib():
    """Open libradcool.so (once).  Raises RadcoolError if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RadcoolError(-4, "libradcool.so is not built; run python -m paper_2505_08855_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        P = ctypes.POINTER
        sig = {
            "rc_default_spec": (i32, [P(TableSpec), i32]),
            "rc_default_opts": (i32, [P(StepOpts)]),
            "rc_build_tables": (i32, [P(TableSpec), vp, P(vp)]),
            "rc_tables_import": (i32, [P(TableSpec), vp, vp, vp, P(vp)]),
            "rc_tables_export": (i32, [vp, vp, vp]),
            "rc_tables_info": (i32, [vp, P(TableSpec), P(i64)]),
            "rc_tables_save": (i32, [vp, ctypes.c_char_p]),
            "rc_tables_load": (i32, [ctypes.c_char_p, vp, P(vp)]),
            "rc_tables_destroy": (i32, [vp]),
            "rc_tables_storage_bytes": (i32, [P(TableSpec), P(ctypes.c_uint64)]),
            "rc_cool_step": (i32, [vp, P(State), i64, dbl, P(StepOpts), P(Out), vp]),
            "rc_cool_step_noalloc": (i32, [vp, P(State), i64, dbl, P(StepOpts), P(Out), vp]),
            "rc_constants": (i32, [vp, i32]),
            "rc_selftest_node_host": (i32, [P(TableSpec), i32, i32, i32, i32, P(dbl)]),
            "rc_selftest_special_host": (i32, [i32, vp, vp, i64]),
            "rc_selftest_step_host": (i32, [P(TableSpec), vp, vp, vp, vp, vp, vp, vp, vp, i64, dbl,
                                            P(StepOpts), vp, vp, vp, vp, vp]),
            "rc_last_error": (ctypes.c_char_p, []),
            "rc_cool_step_backward": (i32, [vp, P(State), i64, dbl, P(StepOpts), P(Fwd), P(Cotangent), P(Grad), vp]),
            "rc_selftest_backward_host": (i32, [P(TableSpec), vp, vp] + [vp] * 12 + [i64, dbl, P(StepOpts)]
                                          + [vp] * 6),
            "rc_cool_step_batched": (i32, [vp, P(State), i64, vp, i32, vp, i32, P(StepOpts), P(Out), vp]),
            "rc_plan_create": (i32, [vp, P(State), i64, vp, i32, vp, i32, P(StepOpts), P(Out), i32, vp, P(vp)]),
            "rc_plan_launch": (i32, [vp, vp]),
            "rc_plan_info": (i32, [vp, P(i32), P(i32), P(dbl)]),
            "rc_plan_destroy": (i32, [vp]),
            "rc_batched_workgroup_items": (i32, [vp, vp, i32, P(i32)]),
            "rc_plan_workgroup_items": (i32, [vp, vp, i32, P(i32)]),
            "rc_disk_inputs": (i32, [vp, vp, vp, vp, i64, P(DiskParams), vp, vp, vp]),
            "rc_rad_pressure_correction": (i32, [vp, vp, vp, i64, dbl, vp, vp, vp]),
            "rc_selftest_disk_host": (i32, [vp, vp, vp, vp, i64, P(DiskParams), vp, vp]),
            "rc_selftest_radp_host": (i32, [vp, vp, vp, i64, dbl, vp, vp]),
            "rc_apply_cooling": (i32, [vp, vp, vp, vp, vp, i64, dbl, P(Coupling), vp, vp]),
            "rc_selftest_coupling_host": (i32, [vp, vp, vp, vp, vp, i64, dbl, P(Coupling), vp]),
            "rc_paper_axes4": (i32, [P(Axes4), i32]),
            "rc_build_table4d": (i32, [P(Axes4), vp, P(vp)]),
            "rc_table4d_import": (i32, [P(Axes4), vp, vp, P(vp)]),
            "rc_table4d_export": (i32, [vp, P(Axes4), vp]),
            "rc_table4d_destroy": (i32, [vp]),
            "rc_rates4d": (i32, [vp, P(State), i64, dbl, vp, vp, vp]),
            "rc_selftest_node4d_host": (i32, [vp, vp, vp, vp, i64, vp]),
            "rc_selftest_rates4d_host": (i32, [P(Axes4), vp, vp, vp, vp, vp, i64, dbl, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code):
    if code != RC_OK:
        raise RadcoolError(code, lib().rc_last_error().decode())


def default_spec(n=64, value_dtype="f32", compton="derived", theta_i_mass="m_p"):
    """Default axes with n nodes each; value_dtype 'f32' or 'bf16' residual
    storage; compton 'derived' or 'literal' (the printed exponent); theta_i_mass
    'm_p' or 'm_e' (the printed theta_i)."""
    s = TableSpec()
    check(lib().rc_default_spec(ctypes.byref(s), n))
    s.value_dtype = VALUE_DTYPES[value_dtype]
    s.compton_exponent = COMPTON[compton]
    s.theta_i_mass = THETA_I_MASS[theta_i_mass]
    return s


def spec_from_axes(cool, coul, ln_lambda=20.0, value_dtype="f32", compton="derived", theta_i_mass="m_p"):
    """Build a TableSpec from two sequences of (n, lo, hi) triples."""
    s = TableSpec()
    for dst, src in ((s.cool, cool), (s.coul, coul)):
        for k, (n, lo, hi) in enumerate(src):
            dst.n[k] = int(n)
            dst.lo[k] = float(lo)
            dst.hi[k] = float(hi)
    s.ln_lambda = ln_lambda
    s.value_dtype = VALUE_DTYPES[value_dtype]
    s.compton_exponent = COMPTON[compton]
    s.theta_i_mass = THETA_I_MASS[theta_i_mass]
    return s


def default_opts(**kw):
    o = StepOpts()
    check(lib().rc_default_opts(ctypes.byref(o)))
    for k, v in kw.items():
        if k == "scheme" and isinstance(v, str):
            v = SCHEMES[v]
        if k == "variant" and isinstance(v, str):
            v = VARIANTS[v]
        if k == "rate_dtype" and isinstance(v, str):
            v = RATE_DTYPES[v]
        setattr(o, k, v)
    return o


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def spec_sizes(spec):
    vc = spec.cool.n[0] * spec.cool.n[1] * spec.cool.n[2]
    vk = spec.coul.n[0] * spec.coul.n[1] * spec.coul.n[2]
    return vc, vk


def storage_bytes(spec):
    """Device bytes the tables of ``spec`` occupy in external storage."""
    n = ctypes.c_uint64()
    check(lib().rc_tables_storage_bytes(ctypes.byref(spec), ctypes.byref(n)))
    return n.value


def _with_storage(spec, storage):
    """A copy of spec pointing at the device tensor ``storage`` (or spec itself)."""
    if storage is None:
        return spec
    s = TableSpec()
    ctypes.pointer(s)[0] = spec
    s.external_storage = storage.data_ptr()
    s.external_bytes = storage.numel() * storage.element_size()
    return s


class Tables:
    """Owning wrapper of an rc_tables handle."""

    def __init__(self, handle, storage=None):
        self._h = ctypes.c_void_p(handle)
        self._storage = storage          # caller-owned device memory the tables live in

    @property
    def handle(self):
        if not self._h:
            raise RadcoolError(-5, "tables already destroyed")
        return self._h

    @staticmethod
    def build(spec=None, stream=None, storage=None):
        """Build tables from the closed forms; ``storage`` (optional) is a
        caller-owned device tensor of at least ``storage_bytes(spec)`` bytes
        that the tables are put into (kept referenced by the returned object)."""
        spec = _with_storage(spec if spec is not None else default_spec(), storage)
        h = ctypes.c_void_p()
        check(lib().rc_build_tables(ctypes.byref(spec), _stream_ptr(stream), ctypes.byref(h)))
        return Tables(h.value, storage)

    @staticmethod
    def from_storage(spec, resid, coeffs, stream=None, storage=None):
        """Create tables from host FP32 residuals (all four tables back to back) and
        FP64 coefficients (4 x 4); ``storage`` as for ``build``."""
        resid = np.ascontiguousarray(resid, dtype=np.float32).ravel()
        coeffs = np.ascontiguousarray(coeffs, dtype=np.float64).ravel()
        vc, vk = spec_sizes(spec)
        if resid.size != 3 * vc + vk or coeffs.size != 16:
            raise ValueError("storage arrays do not match the spec")
        spec = _with_storage(spec, storage)
        h = ctypes.c_void_p()
        check(lib().rc_tables_import(ctypes.byref(spec), resid.ctypes.data_as(ctypes.c_void_p),
                                     coeffs.ctypes.data_as(ctypes.c_void_p), _stream_ptr(stream),
                                     ctypes.byref(h)))
        return Tables(h.value, storage)

    @staticmethod
    def load(path, stream=None):
        h = ctypes.c_void_p()
        check(lib().rc_tables_load(path.encode(), _stream_ptr(stream), ctypes.byref(h)))
        return Tables(h.value)

    def save(self, path):
        check(lib().rc_tables_save(self.handle, path.encode()))

    def info(self):
        spec = TableSpec()
        n = ctypes.c_int64()
        check(lib().rc_tables_info(self.handle, ctypes.byref(spec), ctypes.byref(n)))
        return spec, n.value

    def export(self):
        """(resid float32 [3*vc + vk], coeffs float64 [4, 4]) on the host."""
        spec, n = self.info()
        resid = np.empty(n, dtype=np.float32)
        coeffs = np.empty(16, dtype=np.float64)
        check(lib().rc_tables_export(self.handle, resid.ctypes.data_as(ctypes.c_void_p),
                                     coeffs.ctypes.data_as(ctypes.c_void_p)))
        return resid, coeffs.reshape(4, 4)

    def destroy(self):
        if self._h:
            lib().rc_tables_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _check_out(out, n, opts):
    """Output tensors must match the kernels' element types and the cell count."""
    import torch
    rt = torch.float32 if opts.rate_dtype == RATE_DTYPES["f32"] else torch.float64
    want = {"T_e_new": torch.float64, "T_i_new": torch.float64, "Q_rad": rt, "Q_cc": rt, "status": torch.uint8,
            "Q_brem": torch.float64, "Q_syn": torch.float64, "eta": torch.float64}
    for k, t in out.items():
        if t is None:
            continue
        if k not in want:
            raise ValueError("unknown output %s" % k)
        if t.dtype != want[k] or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
            raise ValueError("output %s must be a contiguous %s HIP tensor of %d elements" % (k, want[k], n))
    return out


def _check_state(state):
    import torch
    ref = state["n_e"]
    for k in ("n_e", "T_e", "T_i", "B", "H", "T_floor_gas"):
        t = state.get(k)
        if t is None and k == "T_floor_gas":
            continue
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != ref.numel():
            raise ValueError("state field %s must be a contiguous float64 HIP tensor of equal length" % k)
    return ref.numel()


def cool_step(tables, state, dt, opts=None, out=None, diagnostics=False, stream=None):
    """One cooling step.  ``state``: dict of float64 device tensors n_e, T_e, T_i, B, H
    and optionally T_floor_gas (per-cell gas-temperature floor, K).

    Returns a dict of output tensors (allocated here unless ``out`` supplies them):
    T_e_new, T_i_new, Q_rad, Q_cc, status (+ Q_brem, Q_syn, eta with diagnostics).
    """
    import torch
    n = _check_state(state)
    opts = opts or default_opts()
    dev = state["n_e"].device
    if out is None:
        rt = torch.float32 if opts.rate_dtype == RATE_DTYPES["f32"] else torch.float64
        out = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("T_e_new", "T_i_new")}
        out.update({k: torch.empty(n, dtype=rt, device=dev) for k in ("Q_rad", "Q_cc")})
        out["status"] = torch.empty(n, dtype=torch.uint8, device=dev)
        if diagnostics:
            for k in ("Q_brem", "Q_syn", "eta"):
                out[k] = torch.empty(n, dtype=torch.float64, device=dev)
    _check_out(out, n, opts)
    st = _state(state)
    o = Out(*[out[k].data_ptr() if out.get(k) is not None else None
              for k in ("T_e_new", "T_i_new", "Q_rad", "Q_cc", "status", "Q_brem", "Q_syn", "eta")])
    check(lib().rc_cool_step(tables.handle, ctypes.byref(st), n, float(dt), ctypes.byref(opts),
                             ctypes.byref(o), _stream_ptr(stream)))
    return out


def cool_step_noalloc(tables, state, dt, out, opts=None, stream=None):
    """rc_cool_step_noalloc: the step of cool_step with no device allocation in
    the library (static scratch, at most NOALLOC_MAX_CELLS cells).  ``out``
    supplies every output tensor (T_e_new, T_i_new, Q_rad, Q_cc, status;
    optionally Q_brem, Q_syn, eta).  Returns ``out``."""
    n = _check_state(state)
    opts = opts or default_opts()
    _check_out(out, n, opts)
    st = _state(state)
    o = _out_struct(out)
    check(lib().rc_cool_step_noalloc(tables.handle, ctypes.byref(st), n, float(dt), ctypes.byref(opts),
                                     ctypes.byref(o), _stream_ptr(stream)))
    return out


def cool_step_backward(tables, state, dt, fwd, cot, opts=None, table_grad=None, stream=None):
    """Vector-Jacobian product of cool_step.  ``fwd``: dict with T_e_new, T_i_new,
    status from the forward call; ``cot``: dict of cotangent tensors (any of
    T_e_new, T_i_new, Q_rad, Q_cc; missing = 0).  Returns a dict of input
    gradients (n_e, T_e, T_i, B, H); if ``table_grad`` (a float64 tensor of
    n_values) is given, table-entry gradients are accumulated into it."""
    import torch
    n = _check_state(state)
    opts = opts or default_opts()
    dev = state["n_e"].device
    g = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("n_e", "T_e", "T_i", "B", "H")}
    st = _state(state)
    fw = Fwd(*[fwd[k].data_ptr() if fwd is not None and fwd.get(k) is not None else None
               for k in ("T_e_new", "T_i_new", "status")])
    ct = Cotangent(*[cot[k].contiguous().data_ptr() if cot.get(k) is not None else None
                     for k in ("T_e_new", "T_i_new", "Q_rad", "Q_cc")])
    gr = Grad(*[g[k].data_ptr() for k in ("n_e", "T_e", "T_i", "B", "H")],
              table_grad.data_ptr() if table_grad is not None else None)
    check(lib().rc_cool_step_backward(tables.handle, ctypes.byref(st), n, float(dt), ctypes.byref(opts),
                                      ctypes.byref(fw), ctypes.byref(ct), ctypes.byref(gr), _stream_ptr(stream)))
    return g


def blocks_to_device(blocks, device):
    """(first_cell, n_cells, state_id) triples -> a device buffer in rc_block layout."""
    import torch
    arr = np.array([tuple(b) for b in blocks], dtype=BLOCK_DTYPE)
    return torch.from_numpy(arr.view(np.uint8).copy()).to(device), len(arr)


def _out_struct(out):
    return Out(*[out[k].data_ptr() if out.get(k) is not None else None
                 for k in ("T_e_new", "T_i_new", "Q_rad", "Q_cc", "status", "Q_brem", "Q_syn", "eta")])


def _alloc_out(n, dev, opts):
    import torch
    rt = torch.float32 if opts.rate_dtype == RATE_DTYPES["f32"] else torch.float64
    out = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("T_e_new", "T_i_new")}
    out.update({k: torch.empty(n, dtype=rt, device=dev) for k in ("Q_rad", "Q_cc")})
    out["status"] = torch.empty(n, dtype=torch.uint8, device=dev)
    return out


def cool_step_batched(tables, state, blocks_dev, n_blocks, dt_per_state, opts=None, out=None, stream=None):
    """Batched step over mesh blocks (device rc_block buffer from blocks_to_device)
    with one dt per accretion state."""
    n = _check_state(state)
    opts = opts or default_opts()
    out = _check_out(out if out is not None else _alloc_out(n, state["n_e"].device, opts), n, opts)
    dts = np.ascontiguousarray(dt_per_state, dtype=np.float64)
    st = _state(state)
    check(lib().rc_cool_step_batched(tables.handle, ctypes.byref(st), n, ctypes.c_void_p(blocks_dev.data_ptr()),
                                     n_blocks, dts.ctypes.data_as(ctypes.c_void_p), dts.size, ctypes.byref(opts),
                                     ctypes.byref(_out_struct(out)), _stream_ptr(stream)))
    return out


def _workgroup_items(fn, handle):
    g = ctypes.c_int32()
    check(fn(handle, None, 0, ctypes.byref(g)))
    items = np.zeros(g.value, dtype=np.uint32)
    check(fn(handle, items.ctypes.data_as(ctypes.c_void_p), g.value, ctypes.byref(g)))
    return items


def batched_workgroup_items(tables):
    """Work items each workgroup of the last cool_step_batched launch on these
    tables took from the queue (waits for the device)."""
    return _workgroup_items(lib().rc_batched_workgroup_items, tables.handle)


class Plan:
    """A captured (hipGraph) launch of the batched step on fixed buffers."""

    def __init__(self, tables, state, blocks_dev, n_blocks, dt_per_state, opts=None, out=None, autotune=True,
                 stream=None):
        n = _check_state(state)
        self.opts = opts or default_opts()
        self.out = _check_out(out if out is not None else _alloc_out(n, state["n_e"].device, self.opts), n,
                              self.opts)
        self._keep = (tables, state, blocks_dev)      # the plan holds pointers into these
        dts = np.ascontiguousarray(dt_per_state, dtype=np.float64)
        st = _state(state)
        h = ctypes.c_void_p()
        check(lib().rc_plan_create(tables.handle, ctypes.byref(st), n, ctypes.c_void_p(blocks_dev.data_ptr()),
                                   n_blocks, dts.ctypes.data_as(ctypes.c_void_p), dts.size, ctypes.byref(self.opts),
                                   ctypes.byref(_out_struct(self.out)), 1 if autotune else 0, _stream_ptr(stream),
                                   ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        check(lib().rc_plan_launch(self._h, _stream_ptr(stream)))
        return self.out

    def info(self):
        b, g, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        check(lib().rc_plan_info(self._h, ctypes.byref(b), ctypes.byref(g), ctypes.byref(ms)))
        return {"block": b.value, "grid": g.value, "tuned_ms": ms.value}

    def workgroup_items(self):
        """Work items each workgroup of the plan's last launch took (waits for the device)."""
        return _workgroup_items(lib().rc_plan_workgroup_items, self._h)

    def destroy(self):
        if self._h:
            lib().rc_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def constants():
    buf = (ctypes.c_double * 8)()
    m = lib().rc_constants(buf, 8)
    return list(buf)[:m]


# ---------------------------------------------------------------- host self-tests


def selftest_node_host(spec, table, i0, i1, i2):
    v = ctypes.c_double()
    check(lib().rc_selftest_node_host(ctypes.byref(spec), table, i0, i1, i2, ctypes.byref(v)))
    return v.value


def selftest_special_host(which, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    check(lib().rc_selftest_special_host(which, x.ctypes.data_as(ctypes.c_void_p),
                                         y.ctypes.data_as(ctypes.c_void_p), x.size))
    return y


def selftest_step_host(spec, resid, coeffs, cells, dt, opts=None):
    """Run the per-cell step on the host CPU (same source as the GPU kernel) on
    tables in storage form (see Tables.from_storage).  Test use only."""
    opts = opts or default_opts()
    resid = np.ascontiguousarray(resid, dtype=np.float32).ravel()
    coeffs = np.ascontiguousarray(coeffs, dtype=np.float64).ravel()
    arrs = [np.ascontiguousarray(cells[k], dtype=np.float64) for k in ("n_e", "T_e", "T_i", "B", "H")]
    n = arrs[0].size
    outs = {k: np.empty(n) for k in ("T_e_new", "T_i_new", "Q_rad", "Q_cc")}
    outs["status"] = np.empty(n, dtype=np.uint8)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    fl = cells.get("T_floor_gas")
    fl = None if fl is None else np.ascontiguousarray(fl, dtype=np.float64)
    check(lib().rc_selftest_step_host(ctypes.byref(spec), P(resid), P(coeffs), *[P(a) for a in arrs],
                                      P(fl) if fl is not None else None, n,
                                      float(dt), ctypes.byref(opts),
                                      P(outs["T_e_new"]), P(outs["T_i_new"]), P(outs["Q_rad"]),
                                      P(outs["Q_cc"]), P(outs["status"])))
    return outs


def selftest_backward_host(spec, resid, coeffs, cells, fwd, cot, dt, opts=None):
    """Run the per-cell adjoint on the host CPU (same source as the GPU kernel).
    Returns (input gradients dict, table gradient array).  Test use only."""
    opts = opts or default_opts()
    resid = np.ascontiguousarray(resid, dtype=np.float32).ravel()
    coeffs = np.ascontiguousarray(coeffs, dtype=np.float64).ravel()
    arrs = [np.ascontiguousarray(cells[k], dtype=np.float64) for k in ("n_e", "T_e", "T_i", "B", "H")]
    n = arrs[0].size
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a is not None else None
    fw = [np.ascontiguousarray(fwd["T_e_new"], dtype=np.float64), np.ascontiguousarray(fwd["T_i_new"], dtype=np.float64),
          np.ascontiguousarray(fwd["status"], dtype=np.uint8)]
    ct = [None if cot.get(k) is None else np.ascontiguousarray(np.broadcast_to(cot[k], (n,)), dtype=np.float64)
          for k in ("T_e_new", "T_i_new", "Q_rad", "Q_cc")]
    g = {k: np.empty(n) for k in ("n_e", "T_e", "T_i", "B", "H")}
    gt = np.zeros(resid.size)
    check(lib().rc_selftest_backward_host(ctypes.byref(spec), P(resid), P(coeffs), *[P(a) for a in arrs],
                                          *[P(a) for a in fw], *[P(a) for a in ct], n, float(dt), ctypes.byref(opts),
                                          *[P(g[k]) for k in ("n_e", "T_e", "T_i", "B", "H")], P(gt)))
    return g, gt


# ---------------------------------------------------------------- upstream inputs and post-processing

TAU_CRIT = 4.6      # e^-tau = 0.01: fewer than 1 % of photons escape unscattered


def disk_params(gamma=5.0 / 3.0, spin=0.9375, h_floor=0.1, r_g=None):
    """Disk parameters (defaults: the paper's runs, M = 10 M_sun)."""
    if r_g is None:
        from . import workloads
        r_g = workloads.R_G
    return DiskParams(gamma, spin, h_floor, r_g)


def disk_inputs(prims, params=None, stream=None):
    """H_th [cm] and T_floor_gas [K] per cell from device tensors rho, P, u, r
    (dict).  Returns a dict of two new tensors."""
    import torch
    params = params or disk_params()
    ref = prims["rho"]
    n = ref.numel()
    for k in ("rho", "P", "u", "r"):
        t = prims[k]
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
            raise ValueError("%s must be a contiguous float64 HIP tensor of equal length" % k)
    out = {k: torch.empty(n, dtype=torch.float64, device=ref.device) for k in ("H_th", "T_floor_gas")}
    check(lib().rc_disk_inputs(*[prims[k].data_ptr() for k in ("rho", "P", "u", "r")], n, ctypes.byref(params),
                               out["H_th"].data_ptr(), out["T_floor_gas"].data_ptr(), _stream_ptr(stream)))
    return out


def rad_pressure_correction(n_e, T_e, H, tau_crit=TAU_CRIT, stream=None):
    """(corrected T_e tensor, uint8 thick flags) for float64 device tensors."""
    import torch
    n = n_e.numel()
    for t in (n_e, T_e, H):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
            raise ValueError("inputs must be contiguous float64 HIP tensors of equal length")
    T = torch.empty_like(T_e)
    thick = torch.empty(n, dtype=torch.uint8, device=T_e.device)
    check(lib().rc_rad_pressure_correction(n_e.data_ptr(), T_e.data_ptr(), H.data_ptr(), n, float(tau_crit),
                                           T.data_ptr(), thick.data_ptr(), _stream_ptr(stream)))
    return T, thick


def selftest_disk_host(rho, P, u, r, params=None):
    """rc_disk_inputs' per-cell code on the host (test use)."""
    params = params or disk_params()
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (rho, P, u, r)]
    H = np.empty_like(a[0])
    Tf = np.empty_like(a[0])
    ptr = lambda v: v.ctypes.data_as(ctypes.c_void_p)
    check(lib().rc_selftest_disk_host(*[ptr(v) for v in a], a[0].size, ctypes.byref(params), ptr(H), ptr(Tf)))
    return H, Tf


def selftest_radp_host(n_e, T_e, H, tau_crit=TAU_CRIT):
    """rc_rad_pressure_correction's per-cell code on the host (test use)."""
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (n_e, T_e, H)]
    T = np.empty_like(a[0])
    thick = np.empty(a[0].size, dtype=np.uint8)
    ptr = lambda v: v.ctypes.data_as(ctypes.c_void_p)
    check(lib().rc_selftest_radp_host(*[ptr(v) for v in a], a[0].size, float(tau_crit), ptr(T), ptr(thick)))
    return T, thick


def _coupling(u_cov, U, sqrt_g, ptr):
    c = Coupling()
    for mu in range(4):
        c.u_cov[mu] = ptr(u_cov[mu])
        c.U[mu] = ptr(U[mu]) if U[mu] is not None else None
    c.sqrt_g = ptr(sqrt_g) if sqrt_g is not None else None
    return c


def apply_cooling(state, fwd, u_cov, U, dt, sqrt_g=None, want_lambda=True, stream=None):
    """Apply a step's cooling to the gas energy-momentum in place:
    U[mu] += -dt sqrt(-g) lambda u_cov[mu].  state: n_e, T_e, T_i; fwd: T_e_new,
    T_i_new; u_cov: four tensors; U: four tensors (or None to skip); all
    contiguous float64 device tensors of one length.  Returns lambda (or None)."""
    import torch
    n = state["n_e"].numel()
    ts = [state["n_e"], state["T_e"], state["T_i"], fwd["T_e_new"], fwd["T_i_new"]] + list(u_cov)
    ts += [t for t in U if t is not None] + ([sqrt_g] if sqrt_g is not None else [])
    for t in ts:
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
            raise ValueError("inputs must be contiguous float64 HIP tensors of equal length")
    lam = torch.empty(n, dtype=torch.float64, device=state["n_e"].device) if want_lambda else None
    c = _coupling(u_cov, U, sqrt_g, lambda t: t.data_ptr())
    check(lib().rc_apply_cooling(state["n_e"].data_ptr(), state["T_e"].data_ptr(), state["T_i"].data_ptr(),
                                 fwd["T_e_new"].data_ptr(), fwd["T_i_new"].data_ptr(), n, float(dt),
                                 ctypes.byref(c), lam.data_ptr() if lam is not None else None,
                                 _stream_ptr(stream)))
    return lam


def selftest_coupling_host(n_e, T_e, T_i, T_e_new, T_i_new, u_cov, U, dt, sqrt_g=None):
    """rc_apply_cooling's per-cell code on host arrays (test use).  Returns
    (new U list, lambda)."""
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (n_e, T_e, T_i, T_e_new, T_i_new)]
    u = [np.ascontiguousarray(v, dtype=np.float64) for v in u_cov]
    Un = [None if v is None else np.array(v, dtype=np.float64, copy=True) for v in U]
    sg = None if sqrt_g is None else np.ascontiguousarray(sqrt_g, dtype=np.float64)
    lam = np.empty_like(a[0])
    ptr = lambda v: v.ctypes.data_as(ctypes.c_void_p).value
    c = _coupling(u, Un, sg, ptr)
    check(lib().rc_selftest_coupling_host(*[ptr(v) for v in a], a[0].size, float(dt), ctypes.byref(c), ptr(lam)))
    return Un, lam


# ---------------------------------------------------------------- the paper's 4-D table layout

def paper_axes4(n=100):
    a = Axes4()
    check(lib().rc_paper_axes4(ctypes.byref(a), n))
    return a


class Table4D:
    """log2 Q_total(H, B, n_e, T_e) in the paper's 4-D layout (comparison layout)."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)

    @staticmethod
    def build(axes=None, stream=None):
        axes = axes if axes is not None else paper_axes4()
        h = ctypes.c_void_p()
        check(lib().rc_build_table4d(ctypes.byref(axes), _stream_ptr(stream), ctypes.byref(h)))
        return Table4D(h.value)

    @staticmethod
    def from_values(axes, values, stream=None):
        v = np.ascontiguousarray(values, dtype=np.float32).ravel()
        if v.size != int(np.prod(list(axes.n))):
            raise ValueError("values do not match the axes")
        h = ctypes.c_void_p()
        check(lib().rc_table4d_import(ctypes.byref(axes), v.ctypes.data_as(ctypes.c_void_p), _stream_ptr(stream),
                                      ctypes.byref(h)))
        return Table4D(h.value)

    @property
    def handle(self):
        if not self._h:
            raise RadcoolError(-5, "4-D table destroyed")
        return self._h

    def export(self):
        a = Axes4()
        check(lib().rc_table4d_export(self.handle, ctypes.byref(a), None))
        v = np.empty(tuple(a.n), dtype=np.float32)
        check(lib().rc_table4d_export(self.handle, None, v.ctypes.data_as(ctypes.c_void_p)))
        return a, v

    def destroy(self):
        if self._h:
            lib().rc_table4d_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def rates4d(table4d, state, T_floor=1.0e6, stream=None):
    """(Q_rad, status) tensors from the 4-D table for a dict of device tensors."""
    import torch
    n = _check_state(state)
    dev = state["n_e"].device
    q = torch.empty(n, dtype=torch.float64, device=dev)
    st = torch.empty(n, dtype=torch.uint8, device=dev)
    s = _state(state)
    check(lib().rc_rates4d(table4d.handle, ctypes.byref(s), n, float(T_floor), q.data_ptr(), st.data_ptr(),
                           _stream_ptr(stream)))
    return q, st


def selftest_node4d_host(H, B, n_e, T):
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (H, B, n_e, T)]
    out = np.empty_like(a[0])
    ptr = lambda v: v.ctypes.data_as(ctypes.c_void_p)
    check(lib().rc_selftest_node4d_host(*[ptr(v) for v in a], a[0].size, ptr(out)))
    return out


def selftest_rates4d_host(axes, values, cells, T_floor=1.0e6):
    v = np.ascontiguousarray(values, dtype=np.float32).ravel()
    a = [np.ascontiguousarray(cells[k], dtype=np.float64) for k in ("n_e", "T_e", "B", "H")]
    q = np.empty_like(a[0])
    st = np.empty(a[0].size, dtype=np.uint8)
    ptr = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    check(lib().rc_selftest_rates4d_host(ctypes.byref(axes), ptr(v), *[ptr(x) for x in a], a[0].size,
                                         float(T_floor), ptr(q), ptr(st)))
    return q, st
