"""ctypes binding of librpa (include/rpa.h): argument marshalling only.

Every step of the RPA hot path runs in the HIP library; this module converts NumPy
arrays (host memory) or torch CUDA tensors (device memory) into the C structures and
raises RpaError on a negative status.  The library must have been built
(``paper_2505_06021_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

RPA_OK, RPA_PENDING = 0, 1
RPA_E_ARG, RPA_E_NOMEM, RPA_E_DEVICE, RPA_E_NOTSPD = -1, -2, -3, -4
RPA_E_UNKNOWN_JOB, RPA_E_INTERNAL, RPA_E_CANCELLED = -5, -6, -7
FP64, FP32, BF16X3, F16X3 = 0, 1, 2, 3
MEM_HOST, MEM_DEVICE = 0, 1

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librpa.so")

EXPORTS = ("rpa_init", "rpa_finalize", "rpa_last_error", "rpa_set_stream", "rpa_chi0", "rpa_chi0_noalloc", "rpa_pi",
           "rpa_trln", "rpa_energy", "rpa_points", "rpa_projector", "rpa_philox_B", "rpa_philox_words",
           "rpa_submit", "rpa_poll", "rpa_get_stats", "rpa_profile", "rpa_profile_read", "rpa_tuned")
KERNEL_KINDS = ("philox", "chi0", "pi", "trln", "other", "chi0_aux")


class RpaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rpa error {code}: {msg}")
        self.code = code


class RpaSystemC(C.Structure):
    _fields_ = [("nk", C.c_int32), ("nq", C.c_int32), ("nocc", C.c_int32), ("nvirt", C.c_int32),
                ("naux", C.c_int32), ("is_complex", C.c_int32), ("memspace", C.c_int32),
                ("kq", C.c_void_p), ("eps_occ", C.c_void_p), ("eps_virt", C.c_void_p),
                ("zeta_k", C.c_void_p), ("zeta_q", C.c_void_p), ("B", C.c_void_p),
                ("philox_seed", C.c_uint64), ("sigma", C.c_double), ("vhalf", C.c_void_p),
                ("nk_occ", C.c_int32), ("nbas", C.c_int32), ("c_occ", C.c_void_p), ("c_virt", C.c_void_p),
                ("S_ao", C.c_void_p), ("eps_d", C.c_double)]


class RpaFreqC(C.Structure):
    _fields_ = [("nw", C.c_int32), ("omega", C.c_void_p), ("weight", C.c_void_p)]


class RpaResultC(C.Structure):
    _fields_ = [("E", C.c_double), ("status", C.c_int32), ("npoints", C.c_int32),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
                ("hbm_bytes", C.c_int64)]


class RpaStatsC(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("hbm_limit", "hbm_in_use", "hbm_high_water", "jobs_submitted",
                                         "jobs_done", "jobs_running", "jobs_queued", "fused_launches",
                                         "fused_groups", "solo_groups")]


_lib = None


def load():
    """Load librpa.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2505_06021_amd.build")
    # torch ships its own HIP runtime; loading it first lets librpa bind to that same
    # runtime (matching soname) instead of a second copy from /opt/rocm, so device
    # pointers and streams from torch are valid inside the library.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, U64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    sig = {
        "rpa_init": [C.POINTER(P), C.c_int, U64],
        "rpa_finalize": [P],
        "rpa_set_stream": [P, P],
        "rpa_chi0": [P, C.POINTER(RpaSystemC), I32, D, C.c_int, P],
        "rpa_chi0_noalloc": [P, C.POINTER(RpaSystemC), I32, D, C.c_int, P],
        "rpa_pi": [P, I32, I32, I32, P, P, P],
        "rpa_trln": [P, I32, I32, I32, I32, P, P],
        "rpa_energy": [P, C.POINTER(RpaSystemC), C.POINTER(RpaFreqC), C.c_int, P, P],
        "rpa_points": [P, C.POINTER(RpaSystemC), I32, P, P, C.c_int, P],
        "rpa_projector": [P, I32, I32, D, I32, P, P],
        "rpa_philox_B": [P, U64, D, I32, I32, I32, I32, I32, I32, I32, I32, P],
        "rpa_philox_words": [P, U64, I32, I32, I32, U64, I64, I32, P],
        "rpa_submit": [P, C.POINTER(RpaSystemC), C.POINTER(RpaFreqC), C.c_int, C.POINTER(U64)],
        "rpa_poll": [P, U64, I32, C.POINTER(RpaResultC), P],
        "rpa_get_stats": [P, C.POINTER(RpaStatsC)],
        "rpa_profile": [P, I32],
        "rpa_profile_read": [P, C.POINTER(RpaKernelTimesC)],
        "rpa_tuned": [C.c_char_p, C.c_int32, C.POINTER(C.c_int32)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.rpa_last_error.argtypes = [P]
    lib.rpa_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def tuned():
    """{shape bucket: configuration name} chosen so far by the FP64 chi0 tuner of this process."""
    lib = load()
    need = C.c_int32(0)
    lib.rpa_tuned(None, 0, C.byref(need))
    buf = C.create_string_buffer(need.value + 1)
    lib.rpa_tuned(buf, need.value + 1, C.byref(need))
    out = {}
    for line in buf.value.decode().splitlines():
        key, cfg = line.split()
        out[key] = cfg
    return out


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()          # torch tensor


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class RpaKernelTimesC(C.Structure):
    _fields_ = [("launches", C.c_int64 * 8), ("ms", C.c_double * 8)]


class _Marshal:
    """A C description of a system plus the arrays it points to (kept alive)."""

    def __init__(self, system, device=False, explicit_B=None):
        self.keep = []
        cplx = bool(system.is_complex)
        vdt = np.complex128 if cplx else np.float64
        B = system.B if explicit_B is None else explicit_B
        if device:
            import torch
            dev = torch.device("cuda", 0)

            def put(x, dt):
                t = torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to(dev)
                self.keep.append(t)
                return t.data_ptr()
            mem = MEM_DEVICE
        else:
            def put(x, dt):
                h = _host(x, dt)
                self.keep.append(h)
                return h.ctypes.data
            mem = MEM_HOST
        s = RpaSystemC()
        s.nk, s.nq, s.nocc, s.nvirt, s.naux = system.nk, system.nq, system.nocc, system.nvirt, system.naux
        s.is_complex = 1 if cplx else 0
        s.memspace = mem
        s.kq = put(system.kq, np.int32)
        s.eps_occ = put(system.eps_occ, np.float64)
        s.eps_virt = put(system.eps_virt, np.float64)
        s.zeta_k = put(system.zeta_k, np.float64)
        s.zeta_q = put(system.zeta_q, np.float64)
        if B is not None and not isinstance(B, np.ndarray):      # a torch tensor already on device
            self.keep.append(B)
            s.B = B.data_ptr()
        else:
            s.B = put(B, vdt) if B is not None else None
        s.philox_seed = system.seed
        s.sigma = system.sigma
        s.vhalf = put(system.vhalf, vdt)
        s.nk_occ = int(np.asarray(system.eps_occ).shape[0])
        s.nbas = int(getattr(system, "nbas", 0))
        if s.nbas > 0:
            if getattr(system, "project_on_device", False):
                # raw KS coefficients and the overlaps: the library applies the projector
                nocc = system.nocc
                s.c_occ = put(np.ascontiguousarray(system.c_raw[:, :, :nocc]), np.complex128)
                s.c_virt = put(np.ascontiguousarray(system.c_raw[:, :, nocc:]), np.complex128)
                s.S_ao = put(system.S_ao, np.complex128)
                s.eps_d = float(system.eps_d)
            else:
                s.c_occ = put(system.c_occ, np.complex128)
                s.c_virt = put(system.c_virt, np.complex128)
        if device:
            import torch
            torch.cuda.synchronize()   # the uploads ran on torch's stream
        self.c = s
        self.freq = RpaFreqC()
        self.om = _host(system.omega, np.float64)
        self.wt = _host(system.weight, np.float64)
        self.freq.nw = len(self.om)
        self.freq.omega = self.om.ctypes.data
        self.freq.weight = self.wt.ctypes.data


class Context:
    """One librpa context on HIP device `device`."""

    def __init__(self, device=0, hbm_limit=0):
        self.lib = load()
        h = C.c_void_p()
        self._check(self.lib.rpa_init(C.byref(h), device, int(hbm_limit)))
        self.h = h

    def _check(self, rc):
        if rc < 0:
            msg = self.lib.rpa_last_error(None)
            raise RpaError(rc, msg.decode() if msg else "")
        return rc

    def close(self):
        if getattr(self, "h", None):
            self._check(self.lib.rpa_finalize(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_stream(self, stream_ptr):
        self._check(self.lib.rpa_set_stream(self.h, stream_ptr))

    # ---- synchronous entry points -------------------------------------------------
    def chi0(self, system, iq, omega, prec=FP64, device=False):
        m = _Marshal(system, device=device)
        dt = np.complex128 if system.is_complex else np.float64
        if device:
            import torch
            out = torch.empty((system.naux, system.naux),
                              dtype=torch.complex128 if system.is_complex else torch.float64,
                              device="cuda:0")
            self._check(self.lib.rpa_chi0(self.h, C.byref(m.c), iq, float(omega), prec, out.data_ptr()))
            return out.cpu().numpy()
        out = np.empty((system.naux, system.naux), dtype=dt)
        self._check(self.lib.rpa_chi0(self.h, C.byref(m.c), iq, float(omega), prec, out.ctypes.data))
        return out

    def chi0_noalloc(self, marshal, iq, omega, out, prec=FP64):
        """rpa_chi0_noalloc on a device-memory system description (a _Marshal made with
        device=True and an explicit B) into the complex device tensor `out`."""
        self._check(self.lib.rpa_chi0_noalloc(self.h, C.byref(marshal.c), iq, float(omega), prec,
                                              out.data_ptr()))
        return out

    def pi(self, vhalf, chi0):
        n = vhalf.shape[0]
        cplx = np.iscomplexobj(vhalf) or np.iscomplexobj(chi0)
        dt = np.complex128 if cplx else np.float64
        v, c = _host(vhalf, dt), _host(chi0, dt)
        out = np.empty((n, n), dtype=dt)
        self._check(self.lib.rpa_pi(self.h, n, int(cplx), MEM_HOST, v.ctypes.data, c.ctypes.data,
                                    out.ctypes.data))
        return out

    def trln(self, pis):
        pis = np.asarray(pis)
        if pis.ndim == 2:
            pis = pis[None]
        cplx = np.iscomplexobj(pis)
        p = _host(pis, np.complex128 if cplx else np.float64)
        out = np.empty(p.shape[0], dtype=np.float64)
        self._check(self.lib.rpa_trln(self.h, p.shape[1], p.shape[0], int(cplx), MEM_HOST,
                                      p.ctypes.data, out.ctypes.data))
        return out

    def energy(self, system, prec=FP64, device=False, marshal=None):
        m = marshal if marshal is not None else _Marshal(system, device=device)
        E = C.c_double()
        eps = np.empty((system.nq, len(system.omega)), dtype=np.float64)
        self._check(self.lib.rpa_energy(self.h, C.byref(m.c), C.byref(m.freq), prec, C.addressof(E),
                                        eps.ctypes.data))
        return E.value, eps

    def points(self, system, iqs, omegas, prec=FP64, device=False, marshal=None):
        m = marshal if marshal is not None else _Marshal(system, device=device)
        iq = _host(iqs, np.int32)
        om = _host(omegas, np.float64)
        out = np.empty(len(iq), dtype=np.float64)
        self._check(self.lib.rpa_points(self.h, C.byref(m.c), len(iq), iq.ctypes.data, om.ctypes.data,
                                        prec, out.ctypes.data))
        return out

    def projector(self, S, eps_d):
        """T(k) of the periodic projector from the overlaps S [nk][nbas][nbas] (host)."""
        Sh = _host(S, np.complex128)
        nk, nbas = Sh.shape[0], Sh.shape[1]
        out = np.empty_like(Sh)
        self._check(self.lib.rpa_projector(self.h, nk, nbas, float(eps_d), MEM_HOST, Sh.ctypes.data,
                                           out.ctypes.data))
        return out

    def philox_B(self, seed, sigma, nk, iq, ik, nocc, nvirt, naux, is_complex=True):
        dt = np.complex128 if is_complex else np.float64
        out = np.empty((nocc, nvirt, naux), dtype=dt)
        self._check(self.lib.rpa_philox_B(self.h, seed, sigma, nk, iq, ik, nocc, nvirt, naux,
                                          int(is_complex), MEM_HOST, out.ctypes.data))
        return out

    def philox_words(self, seed, nk, iq, ik, e0, count):
        out = np.empty((count, 4), dtype=np.uint32)
        self._check(self.lib.rpa_philox_words(self.h, seed, nk, iq, ik, e0, count, MEM_HOST,
                                              out.ctypes.data))
        return out

    # ---- serving --------------------------------------------------------------------
    def submit(self, system, prec=FP64):
        m = _Marshal(system, device=False)
        jid = C.c_uint64()
        self._check(self.lib.rpa_submit(self.h, C.byref(m.c), C.byref(m.freq), prec, C.byref(jid)))
        return jid.value

    def poll(self, job_id, timeout_ms=0, nq=None, nw=None):
        """Returns None while pending, else (result dict, eps grid or None)."""
        r = RpaResultC()
        eps = np.empty(nq * nw, dtype=np.float64) if nq and nw else None
        rc = self.lib.rpa_poll(self.h, job_id, int(timeout_ms), C.byref(r),
                               eps.ctypes.data if eps is not None else None)
        if rc == RPA_PENDING:
            return None
        self._check(rc)
        res = dict(E=r.E, status=r.status, npoints=r.npoints, t_submit=r.t_submit,
                   t_start=r.t_start, t_done=r.t_done, hbm_bytes=r.hbm_bytes)
        return res, (eps.reshape(nq, nw) if eps is not None else None)

    def stats(self):
        s = RpaStatsC()
        self._check(self.lib.rpa_get_stats(self.h, C.byref(s)))
        return {n: getattr(s, n) for n, _ in RpaStatsC._fields_}

    def profile(self, enable=True):
        """Turn per-kernel HIP-event timing on (clearing totals) or off."""
        self._check(self.lib.rpa_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        t = RpaKernelTimesC()
        self._check(self.lib.rpa_profile_read(self.h, C.byref(t)))
        return {k: (t.launches[i], t.ms[i]) for i, k in enumerate(KERNEL_KINDS)}
