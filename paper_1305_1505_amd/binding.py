"""ctypes binding of libpin (include/pin.h): argument marshalling only.

Every ``pin_*`` function here has the C entry point's name and arguments; device buffers are
passed as integer addresses (e.g. ``tensor.data_ptr()``) and streams as integer HIP stream
handles (``torch.cuda.current_stream().cuda_stream``; 0 = the null stream).  A non-OK status
raises :class:`PinError`.  Importing this module loads ``libpin.so`` and raises ImportError if
it has not been built -- there is no fallback path.

:class:`Plan` is a convenience wrapper that allocates outputs as torch tensors on the current
device and calls the same entry points.
"""

import ctypes
import os

# torch's ROCm build carries its own HIP runtime (libamdhip64), which libpin.so also links: load
# torch first so that the process holds one runtime.  Loading libpin first brings in the system
# runtime, and torch's own then finds no GPU.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpin.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1305_1505_amd.build`")
lib = ctypes.CDLL(LIB_PATH)

PIN_OK = 0
PIN_ERR_INVALID_ARG = 1
PIN_ERR_UNSUPPORTED_SIZE = 2
PIN_ERR_OUT_OF_MEMORY = 3
PIN_ERR_DEVICE = 4
PIN_ERR_NOT_READY = 5
PIN_ERR_BUDGET = 6
PIN_ERR_CANCELLED = 7
PIN_ERR_SHUTDOWN = 8
PIN_ERR_TIMEOUT = 9

PIN_FP32 = 0
PIN_FP64 = 1
NEVER = 255


class pin_plan_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("box", ctypes.c_double), ("n_radii", ctypes.c_int),
                ("radii_cells", ctypes.POINTER(ctypes.c_double)), ("sigma8", ctypes.c_double),
                ("gamma", ctypes.c_double), ("ns", ctypes.c_double), ("prec", ctypes.c_int)]


class pin_fragment_params(ctypes.Structure):
    _fields_ = [("f_a", ctypes.c_double), ("f_ra", ctypes.c_double), ("f_s", ctypes.c_double),
                ("f_m", ctypes.c_double), ("f_rm", ctypes.c_double)]


class PinError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{lib.pin_status_string(status).decode()} ({status}): {message}")
        self.status = status


_vp = ctypes.c_void_p
_sig = {
    "pin_size_supported": (ctypes.c_int, [ctypes.c_int]),
    "pin_plan_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(pin_plan_desc), ctypes.POINTER(ctypes.c_size_t)]),
    "pin_plan_validate": (ctypes.c_int, [ctypes.POINTER(pin_plan_desc)]),
    "pin_plan_create": (ctypes.c_int, [ctypes.POINTER(pin_plan_desc), ctypes.POINTER(_vp)]),
    "pin_plan_destroy": (ctypes.c_int, [_vp]),
    "pin_plan_set_radii": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int, _vp]),
    "pin_generate_field": (ctypes.c_int, [_vp, ctypes.c_uint64, _vp, _vp]),
    "pin_collapse_reset": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "pin_collapse_times_range": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp]),
    "pin_collapse_times": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "pin_collapse_times_noalloc": (ctypes.c_int, [ctypes.POINTER(pin_plan_desc), _vp, _vp, _vp, _vp]),
    "pin_deformation_tensor": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp]),
    "pin_plan_velocity_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(pin_plan_desc), ctypes.POINTER(ctypes.c_size_t)]),
    "pin_collapse_reset_v": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "pin_collapse_times_range_v": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp]),
    "pin_collapse_times_v": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "pin_plan_set_growth": (ctypes.c_int, [_vp, ctypes.c_double, _vp]),
    "pin_collapse_redshift": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _vp, _vp]),
    "pin_radius_ladder": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "pin_displacements": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "pin_plan_lpt3_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(pin_plan_desc), ctypes.POINTER(ctypes.c_size_t)]),
    "pin_lpt3_displacement": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "pin_fragment_default_params": (None, [ctypes.POINTER(pin_fragment_params)]),
    "pin_plan_fragment_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(pin_plan_desc), ctypes.POINTER(ctypes.c_size_t)]),
    "pin_fragment": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.POINTER(pin_fragment_params), _vp, _vp,
                                    ctypes.POINTER(ctypes.c_int), _vp]),
    "pin_fragment_catalog": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp]),
    "pin_fragment_mergers": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _vp]),
    "pin_inverse_collapse_time": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _vp, _vp]),
    "pin_kernel_class_count": (ctypes.c_int, []),
    "pin_kernel_class_name": (ctypes.c_char_p, [ctypes.c_int]),
    "pin_plan_set_timing": (ctypes.c_int, [_vp, ctypes.c_int]),
    "pin_plan_kernel_time": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_longlong)]),
    "pin_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "pin_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _check(status, library=None):
    if status != PIN_OK:
        raise PinError(status, (library or lib).pin_last_error().decode())


def make_desc(n, box, radii_cells, sigma8=0.8, gamma=0.21, ns=1.0, prec=PIN_FP32):
    """A pin_plan_desc; the returned object keeps the radii array alive."""
    radii = (ctypes.c_double * len(radii_cells))(*[float(r) for r in radii_cells])
    d = pin_plan_desc(int(n), float(box), len(radii_cells), radii, float(sigma8), float(gamma), float(ns), int(prec))
    d._radii = radii
    return d


def pin_size_supported(n):
    return bool(lib.pin_size_supported(int(n)))


def pin_plan_validate(desc):
    _check(lib.pin_plan_validate(ctypes.byref(desc)))


def pin_plan_workspace_bytes(desc):
    out = ctypes.c_size_t(0)
    _check(lib.pin_plan_workspace_bytes(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def pin_plan_create(desc):
    h = _vp()
    _check(lib.pin_plan_create(ctypes.byref(desc), ctypes.byref(h)))
    return h


def pin_plan_destroy(plan):
    _check(lib.pin_plan_destroy(plan))


def pin_plan_set_radii(plan, radii_cells, stream=0):
    radii = (ctypes.c_double * len(radii_cells))(*[float(r) for r in radii_cells])
    _check(lib.pin_plan_set_radii(plan, radii, len(radii_cells), _vp(stream)))


def pin_generate_field(plan, seed, dk, stream=0):
    _check(lib.pin_generate_field(plan, ctypes.c_uint64(int(seed) & (2 ** 64 - 1)), _vp(dk), _vp(stream)))


def pin_collapse_reset(plan, F, ridx, stream=0):
    _check(lib.pin_collapse_reset(plan, _vp(F), _vp(ridx), _vp(stream)))


def pin_collapse_times_range(plan, dk, F, ridx, r_begin, r_end, stream=0):
    _check(lib.pin_collapse_times_range(plan, _vp(dk), _vp(F), _vp(ridx), int(r_begin), int(r_end), _vp(stream)))


def pin_collapse_times(plan, dk, F, ridx, stream=0):
    _check(lib.pin_collapse_times(plan, _vp(dk), _vp(F), _vp(ridx), _vp(stream)))


def pin_collapse_times_noalloc(desc, dk, F, ridx, stream=0):
    _check(lib.pin_collapse_times_noalloc(ctypes.byref(desc), _vp(dk), _vp(F), _vp(ridx), _vp(stream)))


def pin_plan_velocity_workspace_bytes(desc):
    out = ctypes.c_size_t(0)
    _check(lib.pin_plan_velocity_workspace_bytes(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def pin_collapse_reset_v(plan, F, ridx, vmax, stream=0):
    _check(lib.pin_collapse_reset_v(plan, _vp(F), _vp(ridx), _vp(vmax), _vp(stream)))


def pin_collapse_times_range_v(plan, dk, F, ridx, vmax, r_begin, r_end, stream=0):
    _check(lib.pin_collapse_times_range_v(plan, _vp(dk), _vp(F), _vp(ridx), _vp(vmax), int(r_begin), int(r_end),
                                          _vp(stream)))


def pin_collapse_times_v(plan, dk, F, ridx, vmax, stream=0):
    _check(lib.pin_collapse_times_v(plan, _vp(dk), _vp(F), _vp(ridx), _vp(vmax), _vp(stream)))


def pin_plan_set_growth(plan, omega_m, stream=0):
    _check(lib.pin_plan_set_growth(plan, float(omega_m), _vp(stream)))


def pin_collapse_redshift(plan, F, count, zc, stream=0):
    _check(lib.pin_collapse_redshift(plan, _vp(F), ctypes.c_size_t(int(count)), _vp(zc), _vp(stream)))


def pin_radius_ladder(n, box, r_max_cells, r_min_cells, dex=0.15, gamma=0.21, ns=1.0):
    """The radius ladder as a list (host only): first the length, then the radii."""
    count = ctypes.c_int(0)
    args = (int(n), float(box), float(r_max_cells), float(r_min_cells), float(dex), float(gamma), float(ns))
    _check(lib.pin_radius_ladder(*args, None, 0, ctypes.byref(count)))
    out = (ctypes.c_double * max(count.value, 1))()
    _check(lib.pin_radius_ladder(*args, out, count.value, ctypes.byref(count)))
    return [out[i] for i in range(count.value)]


def pin_deformation_tensor(plan, dk, r, T6, stream=0):
    _check(lib.pin_deformation_tensor(plan, _vp(dk), int(r), _vp(T6), _vp(stream)))


def pin_displacements(plan, dk, psi1, psi2, stream=0):
    _check(lib.pin_displacements(plan, _vp(dk), _vp(psi1 or None), _vp(psi2 or None), _vp(stream)))


def pin_plan_lpt3_workspace_bytes(desc):
    out = ctypes.c_size_t()
    _check(lib.pin_plan_lpt3_workspace_bytes(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def pin_lpt3_displacement(plan, dk, psi3, stream=0):
    _check(lib.pin_lpt3_displacement(plan, _vp(dk), _vp(psi3), _vp(stream)))


def pin_fragment_default_params():
    out = pin_fragment_params()
    lib.pin_fragment_default_params(ctypes.byref(out))
    return out


def pin_plan_fragment_workspace_bytes(desc):
    out = ctypes.c_size_t()
    _check(lib.pin_plan_fragment_workspace_bytes(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def pin_fragment_catalog(plan, ids, n_particles, centre, displacement, capacity, stream=0):
    _check(lib.pin_fragment_catalog(plan, _vp(ids), _vp(n_particles), _vp(centre), _vp(displacement), int(capacity),
                                    _vp(stream)))


def pin_fragment_mergers(plan, f, keep, gone, n_keep, n_gone, capacity, stream=0):
    """Returns the number of mergers (with capacity 0 and all arrays 0: only the count)."""
    c = ctypes.c_int(0)
    _check(lib.pin_fragment_mergers(plan, _vp(f or None), _vp(keep or None), _vp(gone or None), _vp(n_keep or None),
                                    _vp(n_gone or None), int(capacity), ctypes.byref(c), _vp(stream)))
    return c.value


def pin_fragment(plan, F, vmax, f_min, params, label, halo_size, stream=0):
    """Returns the number of halos."""
    nh = ctypes.c_int(0)
    _check(lib.pin_fragment(plan, _vp(F), _vp(vmax), float(f_min), ctypes.byref(params) if params is not None else None,
                            _vp(label), _vp(halo_size or None), ctypes.byref(nh), _vp(stream)))
    return nh.value


def pin_inverse_collapse_time(plan, T6, count, F, stream=0):
    _check(lib.pin_inverse_collapse_time(plan, _vp(T6), ctypes.c_size_t(int(count)), _vp(F), _vp(stream)))


def pin_kernel_class_count():
    return lib.pin_kernel_class_count()


def pin_kernel_class_name(cls):
    return lib.pin_kernel_class_name(int(cls)).decode()


def pin_plan_set_timing(plan, enable):
    _check(lib.pin_plan_set_timing(plan, 1 if enable else 0))


def pin_plan_kernel_time(plan, cls):
    ms = ctypes.c_double(0)
    cnt = ctypes.c_longlong(0)
    _check(lib.pin_plan_kernel_time(plan, int(cls), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def pin_status_string(status):
    return lib.pin_status_string(int(status)).decode()


def pin_last_error():
    return lib.pin_last_error().decode()


class Plan:
    """A plan with torch-tensor conveniences (outputs allocated on the current HIP device)."""

    def __init__(self, n, box, radii_cells, sigma8=0.8, gamma=0.21, ns=1.0, prec=PIN_FP32):
        import torch

        self.torch = torch
        self.n = int(n)
        self.box = float(box)
        self.radii = [float(r) for r in radii_cells]
        self.prec = prec
        self.desc = make_desc(n, box, radii_cells, sigma8, gamma, ns, prec)
        self.handle = pin_plan_create(self.desc)
        self.real = torch.float64 if prec == PIN_FP64 else torch.float32
        self.cplx = torch.complex128 if prec == PIN_FP64 else torch.complex64

    def close(self):
        if self.handle is not None:
            pin_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        return self.torch.cuda.current_stream().cuda_stream

    def empty_spectrum(self):
        n = self.n
        return self.torch.empty((n, n, n // 2 + 1), dtype=self.cplx, device="cuda")

    def generate_field(self, seed, dk=None):
        dk = self.empty_spectrum() if dk is None else dk
        pin_generate_field(self.handle, seed, dk.data_ptr(), self._stream())
        return dk

    def _as_spectrum(self, dk):
        if dk.dtype != self.cplx or not dk.is_cuda or not dk.is_contiguous():
            raise TypeError(f"dk must be a contiguous {self.cplx} CUDA tensor")
        if tuple(dk.shape) != (self.n, self.n, self.n // 2 + 1):
            raise ValueError("dk has the wrong shape")
        return dk

    def collapse_times(self, dk, F=None, ridx=None):
        n = self.n
        dk = self._as_spectrum(dk)
        F = self.torch.empty((n, n, n), dtype=self.real, device="cuda") if F is None else F
        ridx = self.torch.empty((n, n, n), dtype=self.torch.uint8, device="cuda") if ridx is None else ridx
        pin_collapse_times(self.handle, dk.data_ptr(), F.data_ptr(), ridx.data_ptr(), self._stream())
        return F, ridx

    def collapse_reset(self, F, ridx):
        pin_collapse_reset(self.handle, F.data_ptr(), ridx.data_ptr(), self._stream())

    def collapse_times_range(self, dk, F, ridx, r_begin, r_end):
        dk = self._as_spectrum(dk)
        pin_collapse_times_range(self.handle, dk.data_ptr(), F.data_ptr(), ridx.data_ptr(), r_begin, r_end,
                                 self._stream())
        return F, ridx

    def collapse_times_v(self, dk, F=None, ridx=None, vmax=None):
        """(F_max, R_max index, v_max [3, N, N, N]) -- pin_collapse_times_v."""
        n = self.n
        dk = self._as_spectrum(dk)
        F = self.torch.empty((n, n, n), dtype=self.real, device="cuda") if F is None else F
        ridx = self.torch.empty((n, n, n), dtype=self.torch.uint8, device="cuda") if ridx is None else ridx
        vmax = self.torch.empty((3, n, n, n), dtype=self.real, device="cuda") if vmax is None else vmax
        pin_collapse_times_v(self.handle, dk.data_ptr(), F.data_ptr(), ridx.data_ptr(), vmax.data_ptr(), self._stream())
        return F, ridx, vmax

    def collapse_reset_v(self, F, ridx, vmax):
        pin_collapse_reset_v(self.handle, F.data_ptr(), ridx.data_ptr(), vmax.data_ptr(), self._stream())

    def collapse_times_range_v(self, dk, F, ridx, vmax, r_begin, r_end):
        dk = self._as_spectrum(dk)
        pin_collapse_times_range_v(self.handle, dk.data_ptr(), F.data_ptr(), ridx.data_ptr(), vmax.data_ptr(),
                                   r_begin, r_end, self._stream())
        return F, ridx, vmax

    def set_growth(self, omega_m):
        pin_plan_set_growth(self.handle, omega_m, self._stream())

    def collapse_redshift(self, F):
        """z_c for a device tensor of F values (plan precision)."""
        F = F.contiguous()
        z = self.torch.empty_like(F)
        pin_collapse_redshift(self.handle, F.data_ptr(), F.numel(), z.data_ptr(), self._stream())
        return z

    def deformation_tensor(self, dk, r):
        n = self.n
        dk = self._as_spectrum(dk)
        T6 = self.torch.empty((6, n, n, n), dtype=self.real, device="cuda")
        pin_deformation_tensor(self.handle, dk.data_ptr(), r, T6.data_ptr(), self._stream())
        return T6

    def inverse_collapse_time(self, t6):
        """F for a (6, count) tensor array (any float dtype; converted to the plan's precision)."""
        t6 = self.torch.as_tensor(t6).to(device="cuda", dtype=self.real).contiguous()
        count = t6.shape[1]
        F = self.torch.empty((count,), dtype=self.real, device="cuda")
        pin_inverse_collapse_time(self.handle, t6.data_ptr(), count, F.data_ptr(), self._stream())
        return F

    def displacements(self, dk, want_psi1=True, want_psi2=True):
        n = self.n
        dk = self._as_spectrum(dk)
        p1 = self.torch.empty((3, n, n, n), dtype=self.real, device="cuda") if want_psi1 else None
        p2 = self.torch.empty((3, n, n, n), dtype=self.real, device="cuda") if want_psi2 else None
        pin_displacements(self.handle, dk.data_ptr(), p1.data_ptr() if p1 is not None else 0,
                          p2.data_ptr() if p2 is not None else 0, self._stream())
        return p1, p2

    def fragment(self, F, vmax, f_min=1.0, params=None, want_sizes=True):
        """(label int32 [N, N, N], halo_size int32 [N, N, N] or None, number of halos) -- pin_fragment."""
        n = self.n
        label = self.torch.empty((n, n, n), dtype=self.torch.int32, device="cuda")
        sizes = self.torch.empty((n, n, n), dtype=self.torch.int32, device="cuda") if want_sizes else None
        count = pin_fragment(self.handle, F.data_ptr(), vmax.data_ptr(), f_min, params, label.data_ptr(),
                             sizes.data_ptr() if sizes is not None else 0, self._stream())
        return label, sizes, count

    def fragment_catalog(self, n_halos):
        """(ids, n_particles, centre [3, H], displacement [3, H]) of the last fragment() -- pin_fragment_catalog."""
        t = self.torch
        h = max(int(n_halos), 1)
        ids = t.empty(h, dtype=t.int32, device="cuda")
        cnt = t.empty(h, dtype=t.int32, device="cuda")
        centre = t.empty((3, h), dtype=t.float64, device="cuda")
        disp = t.empty((3, h), dtype=t.float64, device="cuda")
        pin_fragment_catalog(self.handle, ids.data_ptr(), cnt.data_ptr(), centre.data_ptr(), disp.data_ptr(), h,
                             self._stream())
        k = int(n_halos)
        return ids[:k], cnt[:k], centre[:, :k], disp[:, :k]

    def fragment_mergers(self):
        """(f, keep, gone, n_keep, n_gone) of the last fragment(), in the order the mergers happened."""
        t = self.torch
        m = pin_fragment_mergers(self.handle, 0, 0, 0, 0, 0, 0, self._stream())
        h = max(m, 1)
        f = t.empty(h, dtype=t.float64, device="cuda")
        ints = [t.empty(h, dtype=t.int32, device="cuda") for _ in range(4)]
        pin_fragment_mergers(self.handle, f.data_ptr(), *[x.data_ptr() for x in ints], h, self._stream())
        return (f[:m],) + tuple(x[:m] for x in ints)

    def lpt3_displacement(self, dk):
        """psi3 (3, N, N, N) at D = 1 in Mpc/h (pin_lpt3_displacement)."""
        n = self.n
        dk = self._as_spectrum(dk)
        p3 = self.torch.empty((3, n, n, n), dtype=self.real, device="cuda")
        pin_lpt3_displacement(self.handle, dk.data_ptr(), p3.data_ptr(), self._stream())
        return p3


# ---------------------------------------------------------------------------------------------
# Serving (pin_serve_*)

class pin_request(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n", ctypes.c_int), ("box", ctypes.c_double),
                ("n_radii", ctypes.c_int), ("radii_cells", ctypes.POINTER(ctypes.c_double)),
                ("want_disp", ctypes.c_int)]


class pin_result(ctypes.Structure):
    _fields_ = [("F", _vp), ("ridx", _vp), ("psi1", _vp), ("psi2", _vp), ("n", ctypes.c_int),
                ("n_radii", ctypes.c_int), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("status", ctypes.c_int)]


class pin_serve_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_double), ("max_slots_per_class", ctypes.c_int),
                ("device", ctypes.c_int), ("prec", ctypes.c_int), ("sigma8", ctypes.c_double),
                ("gamma", ctypes.c_double), ("ns", ctypes.c_double)]


class pin_serve_stats_t(ctypes.Structure):
    _fields_ = [("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double), ("mean_s", ctypes.c_double),
                ("updates_per_s", ctypes.c_double), ("hbm_in_use", ctypes.c_double),
                ("completed", ctypes.c_longlong), ("failed", ctypes.c_longlong),
                ("cancelled", ctypes.c_longlong), ("queued", ctypes.c_longlong),
                ("running", ctypes.c_longlong), ("slots", ctypes.c_longlong)]


_serve_sig = {
    "pin_serve_slot_bytes": (ctypes.c_int, [ctypes.POINTER(pin_serve_config), ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_size_t)]),
    "pin_serve_create": (ctypes.c_int, [ctypes.POINTER(pin_serve_config), ctypes.POINTER(_vp)]),
    "pin_serve_submit": (ctypes.c_int, [_vp, ctypes.POINTER(pin_request), ctypes.POINTER(ctypes.c_uint64)]),
    "pin_serve_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(pin_result)]),
    "pin_serve_wait": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(pin_result)]),
    "pin_serve_cancel": (ctypes.c_int, [_vp, ctypes.c_uint64]),
    "pin_serve_release": (ctypes.c_int, [_vp, ctypes.c_uint64]),
    "pin_serve_stats": (ctypes.c_int, [_vp, ctypes.POINTER(pin_serve_stats_t)]),
    "pin_serve_reset_stats": (ctypes.c_int, [_vp]),
    "pin_serve_destroy": (ctypes.c_int, [_vp]),
}


class ServeAPI:
    """The pin_serve_* calls of one library (libpin.so, or a test double with the same ABI)."""

    def __init__(self, library):
        self.lib = library
        for name, (res, args) in _serve_sig.items():
            f = getattr(library, name)
            f.restype = res
            f.argtypes = args
        library.pin_last_error.restype = ctypes.c_char_p
        library.pin_last_error.argtypes = []

    def check(self, status):
        _check(status, self.lib)

    def pin_serve_slot_bytes(self, cfg, n):
        out = ctypes.c_size_t(0)
        self.check(self.lib.pin_serve_slot_bytes(ctypes.byref(cfg), int(n), ctypes.byref(out)))
        return out.value

    def pin_serve_create(self, cfg):
        h = _vp()
        self.check(self.lib.pin_serve_create(ctypes.byref(cfg), ctypes.byref(h)))
        return h

    def pin_serve_submit(self, srv, req):
        t = ctypes.c_uint64(0)
        self.check(self.lib.pin_serve_submit(srv, ctypes.byref(req), ctypes.byref(t)))
        return t.value

    def pin_serve_poll(self, srv, ticket):
        """(status, pin_result) without raising on NOT_READY or a failed request."""
        out = pin_result()
        st = self.lib.pin_serve_poll(srv, ctypes.c_uint64(ticket), ctypes.byref(out))
        return st, out

    def pin_serve_wait(self, srv, ticket, timeout_s):
        out = pin_result()
        st = self.lib.pin_serve_wait(srv, ctypes.c_uint64(ticket), float(timeout_s), ctypes.byref(out))
        return st, out

    def pin_serve_cancel(self, srv, ticket):
        self.check(self.lib.pin_serve_cancel(srv, ctypes.c_uint64(ticket)))

    def pin_serve_release(self, srv, ticket):
        self.check(self.lib.pin_serve_release(srv, ctypes.c_uint64(ticket)))

    def pin_serve_stats(self, srv):
        out = pin_serve_stats_t()
        self.check(self.lib.pin_serve_stats(srv, ctypes.byref(out)))
        return {k: getattr(out, k) for k, _ in pin_serve_stats_t._fields_}

    def pin_serve_reset_stats(self, srv):
        self.check(self.lib.pin_serve_reset_stats(srv))

    def pin_serve_destroy(self, srv):
        self.check(self.lib.pin_serve_destroy(srv))


def make_request(seed, n, box, radii_cells, want_disp=1):
    radii = (ctypes.c_double * len(radii_cells))(*[float(r) for r in radii_cells])
    r = pin_request(ctypes.c_uint64(int(seed) & (2 ** 64 - 1)), int(n), float(box), len(radii_cells), radii,
                    int(want_disp))
    r._radii = radii
    return r


def make_serve_config(budget_bytes, max_slots_per_class=4, device=0, prec=PIN_FP32, sigma8=0.8, gamma=0.21,
                      ns=1.0):
    return pin_serve_config(float(budget_bytes), int(max_slots_per_class), int(device), int(prec), float(sigma8),
                            float(gamma), float(ns))


serve = ServeAPI(lib)
pin_serve_slot_bytes = serve.pin_serve_slot_bytes
pin_serve_create = serve.pin_serve_create
pin_serve_submit = serve.pin_serve_submit
pin_serve_poll = serve.pin_serve_poll
pin_serve_wait = serve.pin_serve_wait
pin_serve_cancel = serve.pin_serve_cancel
pin_serve_release = serve.pin_serve_release
pin_serve_stats = serve.pin_serve_stats
pin_serve_reset_stats = serve.pin_serve_reset_stats
pin_serve_destroy = serve.pin_serve_destroy
