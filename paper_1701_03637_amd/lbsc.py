"""ctypes binding of the lbsc C ABI (``include/lbsc.h``).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``liblbsc.so``. PyTorch provides device memory and the stream. Importing
this module fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbsc.so")

FP64, FP32S, FP16S, FP16N, FP16NF = 0, 1, 2, 3, 4
FLAG_FP16S_SINK = 1
PSI_RHO, PSI_EXP = 0, 1
SINK_NONE, SINK_ZMAX, SINK_FACES, SINK_SPHERE = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32s": FP32S, "fp16s": FP16S, "fp16n": FP16N, "fp16nf": FP16NF}
SINKS = {"none": SINK_NONE, "zmax": SINK_ZMAX, "faces": SINK_FACES, "sphere": SINK_SPHERE}
STATUS = {0: "ok", -1: "invalid argument", -2: "invalid state", -3: "HIP runtime error",
          -4: "non-finite density", -5: "unsupported"}


class LbscError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lbsc: {STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("wall_z", ctypes.c_int32),
        ("tau", ctypes.c_double * 2),
        ("g", ctypes.c_double),
        ("psi", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("shift", ctypes.c_double * 2),
        ("sink", ctypes.c_int32),
        ("plane_pad", ctypes.c_int32),
        ("rho_h", ctypes.c_double),
        ("sink_radius", ctypes.c_double),
        ("center", ctypes.c_double * 3),
        ("phi_delta", ctypes.c_double * 2),
        ("solid_z", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("wall_rho", ctypes.c_double * 2),
        ("ncomp", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64),
        ("mass", ctypes.c_double * 2),
        ("evaporated", ctypes.c_double),
        ("evap_rate", ctypes.c_double),
        ("momentum", ctypes.c_double * 3),
        ("z_interface", ctypes.c_double),
        ("r_droplet", ctypes.c_double),
        ("nonfinite", ctypes.c_int64),
        ("nonpositive", ctypes.c_int64),
    ]


class Tiles(ctypes.Structure):
    _fields_ = [("nt", ctypes.c_int32), ("tw", ctypes.c_int32), ("th", ctypes.c_int32), ("nzc", ctypes.c_int32),
                ("variant", ctypes.c_int32)]


SYMBOLS = [
    "lbsc_status_string", "lbsc_last_error", "lbsc_version", "lbsc_create", "lbsc_destroy",
    "lbsc_required_bytes", "lbsc_bind", "lbsc_set_stream", "lbsc_init_from_density",
    "lbsc_init_from_populations", "lbsc_set_sink", "lbsc_step", "lbsc_set_graph", "lbsc_set_tiles", "lbsc_get_tiles",
    "lbsc_tune", "lbsc_num_items", "lbsc_read_density", "lbsc_read_observables", "lbsc_read_populations",
    "lbsc_diagnostics", "lbsc_checkpoint_bytes", "lbsc_save", "lbsc_load", "lbsc_selftest",
    "lbsc_stream_copy", "lbsc_bind_static", "lbsc_set_inst_tiles", "lbsc_get_inst_tiles", "lbsc_tune_cache_save",
    "lbsc_tune_cache_load", "lbsc_tune_cache_clear", "lbsc_kernel_hash",
]

_lib = None


def load_library():
    """Loads liblbsc.so; raises ImportError if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1701_03637_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sz = ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "lbsc_status_string": (ctypes.c_char_p, [i32]),
        "lbsc_last_error": (ctypes.c_char_p, [vp]),
        "lbsc_version": (ctypes.c_char_p, []),
        "lbsc_create": (i32, [i32, ctypes.POINTER(Params), ctypes.POINTER(vp)]),
        "lbsc_destroy": (i32, [vp]),
        "lbsc_required_bytes": (i32, [vp, sz, sz]),
        "lbsc_bind": (i32, [vp, vp, vp, vp]),
        "lbsc_bind_static": (i32, [vp, vp, vp]),
        "lbsc_set_stream": (i32, [vp, vp]),
        "lbsc_init_from_density": (i32, [vp, i32, vp, vp]),
        "lbsc_init_from_populations": (i32, [vp, i32, vp]),
        "lbsc_set_sink": (i32, [vp, i32, i32, dbl, dbl]),
        "lbsc_step": (i32, [vp, i64]),
        "lbsc_set_graph": (i32, [vp, i32]),
        "lbsc_set_tiles": (i32, [vp, ctypes.POINTER(Tiles)]),
        "lbsc_get_tiles": (i32, [vp, ctypes.POINTER(Tiles)]),
        "lbsc_tune": (i32, [vp, i32, ctypes.POINTER(Tiles)]),
        "lbsc_num_items": (i32, [vp, ctypes.POINTER(i32)]),
        "lbsc_read_density": (i32, [vp, i32, i32, vp]),
        "lbsc_read_observables": (i32, [vp, i32, vp, vp, vp]),
        "lbsc_read_populations": (i32, [vp, i32, vp]),
        "lbsc_diagnostics": (i32, [vp, i32, ctypes.POINTER(Diag)]),
        "lbsc_checkpoint_bytes": (i32, [vp, sz]),
        "lbsc_save": (i32, [vp, vp]),
        "lbsc_load": (i32, [vp, vp]),
        "lbsc_selftest": (i32, []),
        "lbsc_stream_copy": (i32, [vp, vp, ctypes.c_size_t, vp]),
        "lbsc_set_inst_tiles": (i32, [vp, i32, ctypes.POINTER(Tiles)]),
        "lbsc_get_inst_tiles": (i32, [vp, i32, ctypes.POINTER(Tiles)]),
        "lbsc_tune_cache_save": (i32, [ctypes.c_char_p]),
        "lbsc_tune_cache_load": (i32, [ctypes.c_char_p, ctypes.POINTER(i32)]),
        "lbsc_tune_cache_clear": (None, []),
        "lbsc_kernel_hash": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def make_params(nx, ny, nz, *, wall_z=False, tau=(1.0, 1.0), g=0.9, psi="rho", precision="fp64",
                shift=(0.04, 0.70), sink="none", rho_h=0.04, sink_radius=0.0, center=None,
                phi_delta=(0.66, -0.66), plane_pad=-1, solid_z=0, wall_rho=(0.0, 0.0), flags=0, ncomp=2) -> Params:
    if center is None:
        center = ((nx - 1) / 2, (ny - 1) / 2, (nz - 1) / 2)
    return Params(nx, ny, nz, int(bool(wall_z)), (ctypes.c_double * 2)(*tau), g,
                  PSI_EXP if psi == "exp" else PSI_RHO, PRECISIONS[precision], (ctypes.c_double * 2)(*shift),
                  SINKS[sink], plane_pad, rho_h, sink_radius, (ctypes.c_double * 3)(*center),
                  (ctypes.c_double * 2)(*phi_delta), int(solid_z), int(flags), (ctypes.c_double * 2)(*wall_rho),
                  int(ncomp), 0)


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def tune_cache_save(path: str):
    st = load_library().lbsc_tune_cache_save(path.encode())
    if st != 0:
        raise LbscError(st, f"tune_cache_save: {path}")


def tune_cache_load(path: str) -> int:
    """Adds the cache entries of the loaded library's kernel sources; returns their number."""
    n = ctypes.c_int32()
    st = load_library().lbsc_tune_cache_load(path.encode(), ctypes.byref(n))
    if st != 0:
        raise LbscError(st, f"tune_cache_load: {path}")
    return n.value


def stream_copy(dst: torch.Tensor, src: torch.Tensor):
    """Copies src into dst (same byte size) with the library's streaming kernel
    on torch's current stream."""
    lib = load_library()
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    st = lib.lbsc_stream_copy(_ptr(dst), _ptr(src), nbytes,
                              ctypes.c_void_p(torch.cuda.current_stream(src.device).cuda_stream))
    if st != 0:
        raise LbscError(st, "stream_copy")


# Bytes between the end of the first population buffer and the start of the
# second (a multiple of 256, not of 4 KiB).
_POP_SKEW = (1 << 20) + (1 << 18) + 1280


class Sim:
    """A context of one or more lattice instances stepped together.

    ``params`` is a Params or a list of Params (one per instance). Buffers are
    torch uint8 tensors on ``device``; the stream is torch's current stream.
    """

    def __init__(self, params, device="cuda:0", static_scratch=False):
        lib = load_library()
        self._lib = lib
        plist = params if isinstance(params, (list, tuple)) else [params]
        self.params = list(plist)
        arr = (Params * len(plist))(*plist)
        h = ctypes.c_void_p()
        st = lib.lbsc_create(len(plist), arr, ctypes.byref(h))
        if st != 0:
            raise LbscError(st, "create: parameters refused")
        self._h = h
        self.device = torch.device(device)
        pb, sb = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(lib.lbsc_required_bytes(h, ctypes.byref(pb), ctypes.byref(sb)))
        self.pop_bytes, self.scratch_bytes = pb.value, sb.value
        # FP64 and FP32S: both population buffers come from one allocation,
        # the second starting _POP_SKEW bytes past the (256-byte rounded) end
        # of the first. Buffers a multiple of 256 KiB apart (separate
        # allocations are 2 MiB aligned) ran the 512^3 step at 15.70 ms (FP64)
        # and 8.63 ms (FP32S), skewed at 15.35 and 8.58: a step reads each
        # node's populations from one buffer while it writes the same node's
        # into the other, and equal low address bits map both streams alike
        # onto the HBM channels. The FP16 forms (5.53 against 5.56 ms for
        # FP16N) keep two allocations.
        if plist[0].precision in (FP64, FP32S):
            off = (pb.value + 255) // 256 * 256 + _POP_SKEW
            self._pop_arena = torch.empty(off + pb.value, dtype=torch.uint8, device=self.device)
            self.pop = [self._pop_arena[:pb.value], self._pop_arena[off:off + pb.value]]
        else:
            self.pop = [torch.empty(pb.value, dtype=torch.uint8, device=self.device) for _ in range(2)]
        self._check(lib.lbsc_set_stream(h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)))
        if static_scratch:
            # the library's static scratch array instead of a caller buffer
            self.scratch = None
            with torch.cuda.device(self.device):
                self._check(lib.lbsc_bind_static(h, _ptr(self.pop[0]), _ptr(self.pop[1])))
        else:
            self.scratch = torch.empty(sb.value, dtype=torch.uint8, device=self.device)
            self._check(lib.lbsc_bind(h, _ptr(self.pop[0]), _ptr(self.pop[1]), _ptr(self.scratch)))

    def _check(self, st):
        if st != 0:
            raise LbscError(st, self._lib.lbsc_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lbsc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def ncomp(self, inst=0) -> int:
        return 1 if self.params[inst].ncomp == 1 else 2

    def n(self, inst=0) -> int:
        p = self.params[inst]
        return p.nx * p.ny * p.nz

    def shape(self, inst=0):
        p = self.params[inst]
        return (p.nz, p.ny, p.nx)

    def _dev64(self, a) -> torch.Tensor:
        t = torch.as_tensor(np.ascontiguousarray(a) if isinstance(a, np.ndarray) else a)
        return t.to(device=self.device, dtype=torch.float64).contiguous()

    def init_from_density(self, rho_a, rho_b=None, inst=0):
        """rho_b may be None (it is ignored) with one component."""
        a = self._dev64(rho_a).reshape(-1)
        b = self._dev64(rho_b).reshape(-1) if rho_b is not None else None
        if a.numel() != self.n(inst) or (b is not None and b.numel() != self.n(inst)):
            raise ValueError("density arrays must have nx*ny*nz elements")
        if b is None and self.ncomp(inst) == 2:
            raise ValueError("two components need both density arrays")
        self._check(self._lib.lbsc_init_from_density(self._h, inst, _ptr(a), _ptr(b) if b is not None else None))
        torch.cuda.synchronize(self.device)

    def init_from_populations(self, f, inst=0):
        t = self._dev64(f).reshape(-1)
        if t.numel() != self.ncomp(inst) * 19 * self.n(inst):
            raise ValueError("populations must have ncomp*19*nx*ny*nz elements")
        self._check(self._lib.lbsc_init_from_populations(self._h, inst, _ptr(t)))
        torch.cuda.synchronize(self.device)

    def set_sink(self, kind: str, rho_h: float, radius: float = 0.0, inst=0):
        self._check(self._lib.lbsc_set_sink(self._h, inst, SINKS[kind], rho_h, radius))

    def step(self, n: int = 1):
        self._check(self._lib.lbsc_step(self._h, int(n)))

    def set_graph(self, steps: int):
        self._check(self._lib.lbsc_set_graph(self._h, int(steps)))

    def set_tiles(self, nt=0, tw=0, th=0, nzc=0, variant=0):
        t = Tiles(nt, tw, th, nzc, variant)
        self._check(self._lib.lbsc_set_tiles(self._h, ctypes.byref(t)))

    def tiles(self):
        """(nt, tw, th, nzc, variant) in use; nt and variant resolved."""
        t = Tiles()
        self._check(self._lib.lbsc_get_tiles(self._h, ctypes.byref(t)))
        return (t.nt, t.tw, t.th, t.nzc, t.variant)

    def tune(self, steps: int = 20):
        t = Tiles()
        self._check(self._lib.lbsc_tune(self._h, int(steps), ctypes.byref(t)))
        return (t.nt, t.tw, t.th, t.nzc, t.variant)

    def set_inst_tiles(self, inst, tw=0, th=0, nzc=0):
        t = Tiles(0, tw, th, nzc, 0)
        self._check(self._lib.lbsc_set_inst_tiles(self._h, inst, ctypes.byref(t)))

    def inst_tiles(self, inst):
        """(nt, tw, th, nzc, variant) of instance inst: its own tw, th, nzc
        (0 = the context's) and the context's resolved nt and variant."""
        t = Tiles()
        self._check(self._lib.lbsc_get_inst_tiles(self._h, inst, ctypes.byref(t)))
        return (t.nt, t.tw, t.th, t.nzc, t.variant)

    def num_items(self) -> int:
        v = ctypes.c_int32()
        self._check(self._lib.lbsc_num_items(self._h, ctypes.byref(v)))
        return v.value

    def density(self, comp=0, inst=0) -> torch.Tensor:
        out = torch.empty(self.n(inst), dtype=torch.float64, device=self.device)
        self._check(self._lib.lbsc_read_density(self._h, inst, comp, _ptr(out)))
        return out.reshape(self.shape(inst))

    def observables(self, inst=0):
        n = self.n(inst)
        ra = torch.empty(n, dtype=torch.float64, device=self.device)
        rb = torch.empty(n, dtype=torch.float64, device=self.device)
        u = torch.empty(3 * n, dtype=torch.float64, device=self.device)
        self._check(self._lib.lbsc_read_observables(self._h, inst, _ptr(ra), _ptr(rb), _ptr(u)))
        s = self.shape(inst)
        return ra.reshape(s), rb.reshape(s), u.reshape((3,) + s)

    def populations(self, inst=0) -> torch.Tensor:
        nc = self.ncomp(inst)
        out = torch.empty(nc * 19 * self.n(inst), dtype=torch.float64, device=self.device)
        self._check(self._lib.lbsc_read_populations(self._h, inst, _ptr(out)))
        return out.reshape((nc, 19) + self.shape(inst))

    def diagnostics(self, inst=0, allow_nonfinite=False) -> dict:
        d = Diag()
        st = self._lib.lbsc_diagnostics(self._h, inst, ctypes.byref(d))
        if st != 0 and not (allow_nonfinite and st == -4):
            self._check(st)
        return {
            "step": d.step, "mass": (d.mass[0], d.mass[1]), "evaporated": d.evaporated,
            "evap_rate": d.evap_rate, "momentum": (d.momentum[0], d.momentum[1], d.momentum[2]),
            "z_interface": d.z_interface, "r_droplet": d.r_droplet,
            "nonfinite": d.nonfinite, "nonpositive": d.nonpositive,
        }

    def checkpoint(self) -> torch.Tensor:
        b = ctypes.c_size_t()
        self._check(self._lib.lbsc_checkpoint_bytes(self._h, ctypes.byref(b)))
        blob = torch.empty(b.value, dtype=torch.uint8, device=self.device)
        self._check(self._lib.lbsc_save(self._h, _ptr(blob)))
        return blob

    def restore(self, blob: torch.Tensor):
        self._check(self._lib.lbsc_load(self._h, _ptr(blob)))
