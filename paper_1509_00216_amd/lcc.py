"""Python binding of libmpslcc (ctypes).  Argument marshalling only.

The names follow the C ABI in include/mpslcc.h: create_hamiltonian, build_environments,
apply_heff, solve_local_lcc, ...  Device vectors are torch tensors on the context's device
(PyTorch is used for device memory and streams); every arithmetic step runs in the library.
If the shared library is missing this module raises on import of the library, it never
falls back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpslcc.so")

LCC_FP64, LCC_FP32, LCC_BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": LCC_FP64, "fp32": LCC_FP32, "bf16x3": LCC_BF16X3}
STATUS = {0: "LCC_OK", 1: "LCC_NOT_CONVERGED", -1: "LCC_ERR_ARG", -2: "LCC_ERR_QN", -3: "LCC_ERR_NOT_SPD",
          -4: "LCC_ERR_NAN", -5: "LCC_ERR_OOM", -6: "LCC_ERR_HIP", -7: "LCC_ERR_STATE", -8: "LCC_ERR_NODEV"}
EXPORTS = ["lcc_context_create", "lcc_context_destroy", "lcc_last_error", "lcc_context_synchronize",
           "lcc_create_hamiltonian", "lcc_hamiltonian_destroy", "lcc_hamiltonian_bond_dims",
           "lcc_hamiltonian_channels", "lcc_hamiltonian_site_mpo", "lcc_build_environments",
           "lcc_build_environments_one_site", "lcc_build_transition_environments_one_site", "lcc_env_destroy",
           "lcc_env_layout", "lcc_env_flops", "lcc_apply_heff", "lcc_solve_local_lcc",
           "lcc_env_profile_apply", "lcc_lowest_eigenvalue", "lcc_env_profile_launches", "lcc_batch_create",
           "lcc_batch_destroy", "lcc_batch_solve", "lcc_solve_local_lcc_batched",
           "lcc_context_set_intermediate_limit", "lcc_sweep_create", "lcc_sweep_destroy", "lcc_sweep_env",
           "lcc_sweep_guess", "lcc_sweep_advance", "lcc_sweep_singular_values", "lcc_context_set_tune_cache",
           "lcc_env_autotune", "lcc_context_set_overlap", "lcc_context_set_plan", "lcc_lowest_eigenpair",
           "lcc_lowest_eigenvalue_noalloc", "lcc_build_transition_environments", "lcc_env_input_layout",
           "lcc_env_ket_tensor", "lcc_env_diagonal", "lcc_sweep_retreat", "lcc_sweep_position",
           "lcc_sweep_attach_reference", "lcc_sweep_first_order_rhs", "lcc_sweep_u_expectation",
           "lcc_mps_expectation", "lcc_sweep_split_block", "lcc_sweep_bond", "lcc_sweep_site_tensor"]


class LccError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class HamDesc(C.Structure):
    _fields_ = [("n_orb", C.c_int32), ("n_elec", C.c_int32), ("two_sz", C.c_int32),
                ("h", C.POINTER(C.c_double)), ("eri", C.POINTER(C.c_double)),
                ("u_onsite", C.POINTER(C.c_double)), ("e_const", C.c_double), ("switch_bond", C.c_int32),
                ("site_order", C.POINTER(C.c_int32)), ("orb_class", C.POINTER(C.c_int32)), ("part", C.c_int32)]


class Sector(C.Structure):
    _fields_ = [("n", C.c_int32), ("two_sz", C.c_int32), ("dim", C.c_int32)]


class MpsBlock(C.Structure):
    _fields_ = [("left", C.c_int32), ("s", C.c_int32), ("right", C.c_int32), ("data", C.POINTER(C.c_double))]


class MpsDesc(C.Structure):
    _fields_ = [("n_sites", C.c_int32), ("bond_offsets", C.POINTER(C.c_int32)), ("sectors", C.POINTER(Sector)),
                ("block_offsets", C.POINTER(C.c_int64)), ("blocks", C.POINTER(MpsBlock))]


class LayoutInfo(C.Structure):
    _fields_ = [("n_elements", C.c_int64), ("n_blocks", C.c_int32), ("n_sectors", C.c_int32),
                ("mpo_bond_dim", C.c_int32), ("transition", C.c_int32), ("flops_per_apply", C.c_double)]


class BlockEntry(C.Structure):
    _fields_ = [("left", C.c_int32), ("s1", C.c_int32), ("s2", C.c_int32), ("right", C.c_int32),
                ("offset", C.c_int64), ("ld", C.c_int32), ("rows", C.c_int32), ("cols", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("max_iter", C.c_int32), ("tol", C.c_double),
                ("inner_tol", C.c_double), ("max_outer", C.c_int32), ("replace_every", C.c_int32),
                ("preconditioner", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("outer", C.c_int32), ("applies_fp64", C.c_int32),
                ("applies_low", C.c_int32), ("rel_residual", C.c_double), ("hylleraas", C.c_double),
                ("e2", C.c_double), ("ms_total", C.c_double)]


class LaunchProfile(C.Structure):
    _fields_ = [("phase", C.c_int32), ("kind", C.c_int32), ("tile_m", C.c_int32), ("tile_n", C.c_int32),
                ("n_tiles", C.c_int32), ("packed", C.c_int32), ("flops", C.c_double), ("bytes", C.c_double),
                ("exec_flops", C.c_double), ("ms", C.c_float), ("layout", C.c_int32)]


class TuneInfo(C.Structure):
    _fields_ = [("tile_overhead", C.c_double), ("split_k", C.c_int64), ("candidates", C.c_int32),
                ("launches", C.c_int32), ("packed_launches", C.c_int32), ("from_cache", C.c_int32),
                ("p2_order", C.c_int32), ("t_colmajor", C.c_int32), ("ms_before", C.c_float), ("ms_after", C.c_float)]


class SiteBlock(C.Structure):
    _fields_ = [("left", C.c_int32), ("s", C.c_int32), ("right", C.c_int32), ("rows", C.c_int32),
                ("cols", C.c_int32), ("offset", C.c_int64)]


class SweepInfo(C.Structure):
    _fields_ = [("site", C.c_int32), ("kept", C.c_int32), ("n_singular", C.c_int32), ("reserved", C.c_int32),
                ("discarded_weight", C.c_double), ("largest_discarded", C.c_double), ("ms_svd", C.c_float),
                ("ms_env", C.c_float), ("ms_guess", C.c_float), ("ms_total", C.c_float)]


_lib = None


def library() -> C.CDLL:
    """Load libmpslcc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1509_00216_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "lcc_context_create": (C.c_int32, [C.c_int32, P, C.POINTER(P)]),
        "lcc_context_destroy": (None, [P]),
        "lcc_last_error": (C.c_char_p, [P]),
        "lcc_context_synchronize": (C.c_int32, [P]),
        "lcc_create_hamiltonian": (C.c_int32, [P, C.POINTER(HamDesc), C.POINTER(P)]),
        "lcc_hamiltonian_destroy": (None, [P]),
        "lcc_hamiltonian_bond_dims": (C.c_int32, [P, C.POINTER(C.c_int32)]),
        "lcc_hamiltonian_channels": (C.c_int32, [P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "lcc_hamiltonian_site_mpo": (C.c_int32, [P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                                 C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
        "lcc_build_environments": (C.c_int32, [P, P, C.POINTER(MpsDesc), C.c_int32, C.POINTER(P)]),
        "lcc_build_environments_one_site": (C.c_int32, [P, P, C.POINTER(MpsDesc), C.c_int32, C.POINTER(P)]),
        "lcc_build_transition_environments_one_site": (C.c_int32, [P, P, C.POINTER(MpsDesc), C.POINTER(MpsDesc),
                                                                   C.c_int32, C.POINTER(P)]),
        "lcc_env_destroy": (None, [P]),
        "lcc_env_layout": (C.c_int32, [P, C.POINTER(LayoutInfo), C.POINTER(BlockEntry)]),
        "lcc_env_input_layout": (C.c_int32, [P, C.POINTER(LayoutInfo), C.POINTER(BlockEntry)]),
        "lcc_env_ket_tensor": (C.c_int32, [P, P]),
        "lcc_env_diagonal": (C.c_int32, [P, P]),
        "lcc_build_transition_environments": (C.c_int32, [P, P, C.POINTER(MpsDesc), C.POINTER(MpsDesc), C.c_int32,
                                                          C.POINTER(P)]),
        "lcc_env_flops": (C.c_int32, [P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "lcc_apply_heff": (C.c_int32, [P, C.c_int32, P, P]),
        "lcc_solve_local_lcc": (C.c_int32, [P, C.POINTER(SolveOpts), P, C.c_double, P, P, C.POINTER(SolveInfo)]),
        "lcc_env_profile_apply": (C.c_int32, [P, C.c_int32, P, P, C.c_int32, C.POINTER(C.c_float),
                                              C.POINTER(C.c_float)]),
        "lcc_lowest_eigenvalue": (C.c_int32, [P, C.c_int32, C.c_uint64, C.POINTER(C.c_double),
                                              C.POINTER(C.c_double)]),
        "lcc_lowest_eigenvalue_noalloc": (C.c_int32, [P, C.c_int32, C.c_uint64, C.POINTER(C.c_double),
                                                      C.POINTER(C.c_double)]),
        "lcc_lowest_eigenpair": (C.c_int32, [P, C.c_int32, C.c_int32, C.c_double, C.c_uint64, P,
                                             C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "lcc_env_profile_launches": (C.c_int32, [P, C.c_int32, P, P, C.c_int32, C.POINTER(C.c_int32),
                                                 C.POINTER(LaunchProfile)]),
        "lcc_batch_create": (C.c_int32, [P, C.c_int32, C.POINTER(P), C.POINTER(P)]),
        "lcc_context_set_intermediate_limit": (C.c_int32, [P, C.c_int64]),
        "lcc_context_set_tune_cache": (C.c_int32, [P, C.c_char_p]),
        "lcc_context_set_overlap": (C.c_int32, [P, C.c_int32]),
        "lcc_context_set_plan": (C.c_int32, [P, C.c_double, C.c_int64, C.c_int32, C.c_int32]),
        "lcc_env_autotune": (C.c_int32, [P, C.c_int32, C.c_int32, C.POINTER(TuneInfo)]),
        "lcc_sweep_create": (C.c_int32, [P, P, C.POINTER(MpsDesc), C.c_int32, C.POINTER(P)]),
        "lcc_sweep_destroy": (None, [P]),
        "lcc_sweep_env": (C.c_int32, [P, C.POINTER(P)]),
        "lcc_sweep_guess": (C.c_int32, [P, P]),
        "lcc_sweep_advance": (C.c_int32, [P, P, C.c_int32, C.POINTER(SweepInfo)]),
        "lcc_sweep_singular_values": (C.c_int32, [P, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
        "lcc_sweep_retreat": (C.c_int32, [P, P, C.c_int32, C.POINTER(SweepInfo)]),
        "lcc_sweep_position": (C.c_int32, [P, C.POINTER(C.c_int32)]),
        "lcc_sweep_attach_reference": (C.c_int32, [P, P, P, C.POINTER(MpsDesc)]),
        "lcc_sweep_first_order_rhs": (C.c_int32, [P, C.c_double, P, P, C.POINTER(C.c_double)]),
        "lcc_sweep_u_expectation": (C.c_int32, [P, P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "lcc_mps_expectation": (C.c_int32, [P, P, C.POINTER(MpsDesc), C.c_int32, C.POINTER(C.c_double)]),
        "lcc_sweep_split_block": (C.c_int32, [P, P, C.c_int32, C.POINTER(SweepInfo)]),
        "lcc_sweep_bond": (C.c_int32, [P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(Sector)]),
        "lcc_sweep_site_tensor": (C.c_int32, [P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                              C.POINTER(SiteBlock), C.POINTER(C.c_double)]),
        "lcc_batch_destroy": (None, [P]),
        "lcc_batch_solve": (C.c_int32, [P, C.POINTER(SolveOpts), C.POINTER(P), C.POINTER(C.c_double), C.POINTER(P),
                                        C.POINTER(P), C.POINTER(SolveInfo)]),
        "lcc_solve_local_lcc_batched": (C.c_int32, [C.c_int32, C.POINTER(P), C.POINTER(SolveOpts), C.POINTER(P),
                                                    C.POINTER(C.c_double), C.POINTER(P), C.POINTER(P),
                                                    C.POINTER(SolveInfo)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(code, ctx=None, allow=(0,)):
    if code in allow:
        return code
    msg = library().lcc_last_error(ctx)
    raise LccError(code, msg.decode() if msg else "")


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _tensor_ptr(t, dtype_name: str, n: int):
    import torch
    want = {"fp64": torch.float64, "fp32": torch.float32}[dtype_name]
    if t.dtype != want or not t.is_contiguous() or t.numel() != n or t.device.type != "cuda":
        raise ValueError(f"expected a contiguous {want} CUDA tensor of {n} elements, got "
                         f"{t.dtype} {tuple(t.shape)} on {t.device}")
    return C.c_void_p(t.data_ptr())


class Context:
    """lcc_context on a device (or host-only with device=-1)."""

    def __init__(self, device: int = 0, stream=None):
        lib = library()
        h = C.c_void_p()
        s = None
        if device >= 0:
            import torch
            if stream is None:
                stream = torch.cuda.current_stream(device)
            s = C.c_void_p(stream.cuda_stream) if stream.cuda_stream else None
        _check(lib.lcc_context_create(device, s, C.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            library().lcc_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def synchronize(self):
        _check(library().lcc_context_synchronize(self.handle), self.handle)

    def set_intermediate_limit(self, nbytes: int):
        _check(library().lcc_context_set_intermediate_limit(self.handle, int(nbytes)), self.handle)

    def set_overlap(self, side_streams: int):
        """Side streams for the independent launches of one GEMM phase (0 = in order)."""
        _check(library().lcc_context_set_overlap(self.handle, int(side_streams)), self.handle)

    def set_plan(self, tile_overhead: float = 2048.0, split_k: int = 2048, p2_order: int = 0, t_colmajor: int = 2):
        """Planner parameters of environments built afterwards (when no tuning-cache entry applies)."""
        _check(library().lcc_context_set_plan(self.handle, float(tile_overhead), int(split_k), int(p2_order),
                                              int(t_colmajor)), self.handle)

    def set_tune_cache(self, path):
        """Autotuning results file (read when environments are built, appended by autotune)."""
        _check(library().lcc_context_set_tune_cache(self.handle, None if path is None else str(path).encode()),
               self.handle)

    def create_hamiltonian(self, spec: dict, switch_bond: int = -1) -> "Hamiltonian":
        return create_hamiltonian(self, spec, switch_bond)

    def build_environments(self, ham: "Hamiltonian", mps: dict, site: int | None = None) -> "Env":
        return build_environments(self, ham, mps, site)

    def build_environments_one_site(self, ham: "Hamiltonian", mps: dict, site: int | None = None) -> "Env":
        return build_environments_one_site(self, ham, mps, site)


def context_create(device: int = 0, stream=None) -> Context:
    return Context(device, stream)


class Hamiltonian:
    def __init__(self, handle, ctx, n_orb):
        self.handle = handle
        self.ctx = ctx
        self.n_orb = n_orb

    def close(self):
        if self.handle:
            library().lcc_hamiltonian_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bond_dims(self) -> np.ndarray:
        out = np.zeros(self.n_orb + 1, dtype=np.int32)
        _check(library().lcc_hamiltonian_bond_dims(self.handle, out.ctypes.data_as(C.POINTER(C.c_int32))))
        return out

    def channels(self, bond: int):
        D = int(self.bond_dims()[bond])
        dn = np.zeros(D, dtype=np.int32)
        dz = np.zeros(D, dtype=np.int32)
        _check(library().lcc_hamiltonian_channels(self.handle, bond, dn.ctypes.data_as(C.POINTER(C.c_int32)),
                                                  dz.ctypes.data_as(C.POINTER(C.c_int32))))
        return dn, dz

    def site_mpo(self, site: int):
        lib = library()
        cnt = C.c_int64(0)
        _check(lib.lcc_hamiltonian_site_mpo(self.handle, site, C.byref(cnt), None, None, None))
        n = cnt.value
        wi = np.zeros(n, dtype=np.int32)
        wo = np.zeros(n, dtype=np.int32)
        m = np.zeros((n, 4, 4))
        _check(lib.lcc_hamiltonian_site_mpo(self.handle, site, C.byref(cnt), wi.ctypes.data_as(C.POINTER(C.c_int32)),
                                            wo.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(m)))
        return wi, wo, m


def create_hamiltonian(ctx: Context | None, spec: dict, switch_bond: int = -1, site_order=None) -> Hamiltonian:
    """spec: n_orb, n_elec, two_sz, h, eri or None, u or None, e_const, and optionally orb_class
    (0 core, 1 active, 2 virtual per orbital) with part (0 H, 1 H0, 2 U)."""
    n = spec["n_orb"]
    h = np.ascontiguousarray(spec["h"], dtype=np.float64)
    eri = None if spec.get("eri") is None else np.ascontiguousarray(spec["eri"], dtype=np.float64)
    u = None if spec.get("u") is None else np.ascontiguousarray(spec["u"], dtype=np.float64)
    order = None if site_order is None else np.ascontiguousarray(site_order, dtype=np.int32)
    cls = None if spec.get("orb_class") is None else np.ascontiguousarray(spec["orb_class"], dtype=np.int32)
    ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32)) if a is not None else None
    d = HamDesc(n, spec["n_elec"], spec["two_sz"], _dptr(h), _dptr(eri) if eri is not None else None,
                _dptr(u) if u is not None else None, float(spec.get("e_const", 0.0)), switch_bond,
                ip(order), ip(cls), int(spec.get("part", 0)))
    out = C.c_void_p()
    ch = ctx.handle if ctx is not None else None
    _check(library().lcc_create_hamiltonian(ch, C.byref(d), C.byref(out)), ch)
    return Hamiltonian(out, ctx, n)


def _mps_desc(mps: dict):
    """Marshal a workloads-style MPS dict into lcc_mps_desc (keeps the arrays alive)."""
    K = mps["n_sites"]
    bond_off = np.zeros(K + 2, dtype=np.int32)
    secs = []
    for j, bond in enumerate(mps["bonds"]):
        secs.extend(bond)
        bond_off[j + 1] = len(secs)
    bond_off[K + 1] = len(secs)
    sectors = (Sector * max(1, len(secs)))(*[Sector(int(n), int(z), int(d)) for n, z, d in secs])
    keep = []
    blocks = []
    blk_off = np.zeros(K + 1, dtype=np.int64)
    for j, site in enumerate(mps["sites"]):
        for il, s, ir, a in site:
            arr = np.ascontiguousarray(a, dtype=np.float64)
            keep.append(arr)
            blocks.append(MpsBlock(int(il), int(s), int(ir), _dptr(arr)))
        blk_off[j + 1] = len(blocks)
    barr = (MpsBlock * max(1, len(blocks)))(*blocks)
    desc = MpsDesc(K, bond_off.ctypes.data_as(C.POINTER(C.c_int32)), sectors,
                   blk_off.ctypes.data_as(C.POINTER(C.c_int64)), barr)
    return desc, (bond_off, sectors, blk_off, barr, keep)


class Env:
    """Environments + plan of one two-site block; vectors use `layout()`."""

    def __init__(self, handle, ctx: Context):
        self.handle = handle
        self.ctx = ctx
        info = LayoutInfo()
        _check(library().lcc_env_layout(self.handle, C.byref(info), None))
        self.n = int(info.n_elements)
        self.n_blocks = int(info.n_blocks)
        self.n_sectors = int(info.n_sectors)
        self.mpo_bond_dim = int(info.mpo_bond_dim)
        self.transition = bool(info.transition)
        self.flops_per_apply = float(info.flops_per_apply)
        arr = (BlockEntry * max(1, self.n_blocks))()
        _check(library().lcc_env_layout(self.handle, C.byref(info), arr))
        self.blocks = {(b.left, b.s1, b.s2, b.right): (b.offset, b.ld, b.rows, b.cols)
                       for b in arr[: self.n_blocks]}
        # input side (the ket's two-site tensor of a transition operator; else the same layout)
        _check(library().lcc_env_input_layout(self.handle, C.byref(info), None))
        self.n_in = int(info.n_elements)
        arr = (BlockEntry * max(1, int(info.n_blocks)))()
        _check(library().lcc_env_input_layout(self.handle, C.byref(info), arr))
        self.blocks_in = {(b.left, b.s1, b.s2, b.right): (b.offset, b.ld, b.rows, b.cols)
                          for b in arr[: int(info.n_blocks)]}

    def close(self):
        if self.handle:
            library().lcc_env_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def flops(self):
        a, b = C.c_double(), C.c_double()
        _check(library().lcc_env_flops(self.handle, C.byref(a), C.byref(b)))
        return a.value, b.value

    # -- marshalling between {(a, s1, s2, b): block} dicts and flat vectors
    def pack(self, vec: dict) -> np.ndarray:
        out = np.zeros(self.n)
        for key, (off, ld, rows, cols) in self.blocks.items():
            blk = vec.get(key)
            if blk is None:
                continue
            idx = off + np.arange(rows)[:, None] * ld + np.arange(cols)[None, :]
            out[idx] = blk
        return out

    def unpack(self, flat: np.ndarray) -> dict:
        out = {}
        for key, (off, ld, rows, cols) in self.blocks.items():
            idx = off + np.arange(rows)[:, None] * ld + np.arange(cols)[None, :]
            out[key] = np.asarray(flat)[idx]
        return out

    def pack_in(self, vec: dict) -> np.ndarray:
        """pack() for the input side (the ket's layout of a transition operator)."""
        out = np.zeros(self.n_in)
        for key, (off, ld, rows, cols) in self.blocks_in.items():
            blk = vec.get(key)
            if blk is None:
                continue
            idx = off + np.arange(rows)[:, None] * ld + np.arange(cols)[None, :]
            out[idx] = blk
        return out

    def ket_tensor(self, x):
        """lcc_env_ket_tensor: the ket's two-site tensor of a transition operator into x (FP64, input layout)."""
        _check(library().lcc_env_ket_tensor(self.handle, _tensor_ptr(x, "fp64", self.n_in)), self.ctx.handle)

    def apply_heff(self, x, y, precision: str = "fp64"):
        dt = "fp64" if precision == "fp64" else "fp32"
        _check(library().lcc_apply_heff(self.handle, PRECISIONS[precision], _tensor_ptr(x, dt, self.n_in),
                                        _tensor_ptr(y, dt, self.n)), self.ctx.handle)

    def profile_apply(self, x, y, precision: str = "fp64", reps: int = 10):
        """Mean milliseconds of (phase 1, phase 2) of H_eff x, timed with HIP events."""
        dt = "fp64" if precision == "fp64" else "fp32"
        a, b = C.c_float(), C.c_float()
        _check(library().lcc_env_profile_apply(self.handle, PRECISIONS[precision], _tensor_ptr(x, dt, self.n),
                                               _tensor_ptr(y, dt, self.n), reps, C.byref(a), C.byref(b)),
               self.ctx.handle)
        return a.value, b.value

    def profile_launches(self, x, y, precision: str = "fp64", reps: int = 10) -> list:
        """Per-launch mean duration (HIP events) with the launch's algorithmic flops and bytes."""
        dt = "fp64" if precision == "fp64" else "fp32"
        lib = library()
        cnt = C.c_int32(0)
        _check(lib.lcc_env_profile_launches(self.handle, PRECISIONS[precision], None, None, 1, C.byref(cnt), None),
               self.ctx.handle)
        arr = (LaunchProfile * cnt.value)()
        _check(lib.lcc_env_profile_launches(self.handle, PRECISIONS[precision], _tensor_ptr(x, dt, self.n),
                                            _tensor_ptr(y, dt, self.n), reps, C.byref(cnt), arr), self.ctx.handle)
        return [{"phase": a.phase, "kind": "gemm" if a.kind == 0 else "reduce", "tile": (a.tile_m, a.tile_n),
                 "n_tiles": a.n_tiles, "packed": bool(a.packed), "flops": a.flops, "bytes": a.bytes,
                 "exec_flops": a.exec_flops, "ms": a.ms, "a_kmajor": bool(a.layout & 1), "b_colmajor": bool(a.layout & 2)}
                for a in arr[: cnt.value]]

    def autotune(self, precision: str = "fp32", reps: int = 3) -> dict:
        """Time the planner candidates and both GEMM kernels per launch; keep the fastest."""
        info = TuneInfo()
        _check(library().lcc_env_autotune(self.handle, PRECISIONS[precision], reps, C.byref(info)), self.ctx.handle)
        return {"tile_overhead": info.tile_overhead, "split_k": info.split_k, "p2_order": info.p2_order,
                "t_colmajor": info.t_colmajor,
                "candidates": info.candidates,
                "launches": info.launches, "packed_launches": info.packed_launches,
                "from_cache": bool(info.from_cache), "ms_before": info.ms_before, "ms_after": info.ms_after}

    def lowest_eigenvalue(self, steps: int = 60, seed: int = 1):
        th, res = C.c_double(), C.c_double()
        _check(library().lcc_lowest_eigenvalue(self.handle, steps, seed, C.byref(th), C.byref(res)),
               self.ctx.handle)
        return th.value, res.value

    def lowest_eigenvalue_noalloc(self, steps: int = 60, seed: int = 1):
        """lcc_lowest_eigenvalue_noalloc: the Krylov basis in the library's fixed device array."""
        th, res = C.c_double(), C.c_double()
        _check(library().lcc_lowest_eigenvalue_noalloc(self.handle, steps, seed, C.byref(th), C.byref(res)),
               self.ctx.handle)
        return th.value, res.value

    def lowest_eigenpair(self, x, steps: int = 40, max_restarts: int = 20, tol: float = 1e-10, seed: int = 1) -> dict:
        """Lowest eigenpair of H_eff; x (FP64 device tensor) holds the start vector (zeros: random)
        on entry and the unit Ritz vector on return."""
        th, res = C.c_double(), C.c_double()
        code = library().lcc_lowest_eigenpair(self.handle, steps, max_restarts, tol, seed,
                                              _tensor_ptr(x, "fp64", self.n), C.byref(th), C.byref(res))
        _check(code, self.ctx.handle, allow=(0, 1))
        return {"status": STATUS[code], "theta": th.value, "residual": res.value}

    def diagonal(self, d):
        """lcc_env_diagonal: diag(H_eff) into d (FP64 device tensor)."""
        _check(library().lcc_env_diagonal(self.handle, _tensor_ptr(d, "fp64", self.n)), self.ctx.handle)

    def solve_local_lcc(self, b, e0: float, x, v=None, precision: str = "fp64", tol: float = 1e-10,
                        max_iter: int = 1000, inner_tol: float = 0.0, max_outer: int = 20,
                        replace_every: int = 50, preconditioner: str = "none") -> dict:
        opts = SolveOpts(PRECISIONS[precision], max_iter, tol, inner_tol, max_outer, replace_every,
                         {"none": 0, "jacobi": 1}[preconditioner])
        info = SolveInfo()
        code = library().lcc_solve_local_lcc(self.handle, C.byref(opts), _tensor_ptr(b, "fp64", self.n),
                                             float(e0), _tensor_ptr(v, "fp64", self.n) if v is not None else None,
                                             _tensor_ptr(x, "fp64", self.n), C.byref(info))
        _check(code, self.ctx.handle, allow=(0, 1))
        return {"status": STATUS[code], "iterations": info.iterations, "outer": info.outer,
                "applies_fp64": info.applies_fp64, "applies_low": info.applies_low,
                "rel_residual": info.rel_residual, "hylleraas": info.hylleraas, "e2": info.e2,
                "ms_total": info.ms_total}


def build_environments(ctx: Context, ham: Hamiltonian, mps: dict, site: int | None = None) -> Env:
    if site is None:
        site = mps["center"]
    desc, keep = _mps_desc(mps)
    out = C.c_void_p()
    _check(library().lcc_build_environments(ctx.handle, ham.handle, C.byref(desc), site, C.byref(out)), ctx.handle)
    del keep
    return Env(out, ctx)


def build_environments_one_site(ctx: Context, ham: Hamiltonian, mps: dict, site: int | None = None) -> Env:
    """lcc_build_environments_one_site: the local problem of the one site tensor at `site`
    (default mps['center']); vector blocks are keyed (a, s, 0, b)."""
    if site is None:
        site = mps["center"]
    desc, keep = _mps_desc(mps)
    out = C.c_void_p()
    _check(library().lcc_build_environments_one_site(ctx.handle, ham.handle, C.byref(desc), site, C.byref(out)),
           ctx.handle)
    del keep
    return Env(out, ctx)


def build_transition_environments(ctx: Context, ham: Hamiltonian, bra: dict, ket: dict, site: int | None = None) -> Env:
    """lcc_build_transition_environments: <bra| H |ket> with the bra's two-site block cut out."""
    if site is None:
        site = bra["center"]
    bd, keep_b = _mps_desc(bra)
    kd, keep_k = _mps_desc(ket)
    out = C.c_void_p()
    _check(library().lcc_build_transition_environments(ctx.handle, ham.handle, C.byref(bd), C.byref(kd), site,
                                                       C.byref(out)), ctx.handle)
    del keep_b, keep_k
    return Env(out, ctx)


def build_transition_environments_one_site(ctx: Context, ham: Hamiltonian, bra: dict, ket: dict,
                                           site: int | None = None) -> Env:
    """lcc_build_transition_environments_one_site: <bra| H |ket> with the bra's site tensor at
    `site` (default bra['center']) cut out; vector blocks keyed (a, s, 0, b)."""
    if site is None:
        site = bra["center"]
    bd, keep_b = _mps_desc(bra)
    kd, keep_k = _mps_desc(ket)
    out = C.c_void_p()
    _check(library().lcc_build_transition_environments_one_site(ctx.handle, ham.handle, C.byref(bd), C.byref(kd), site,
                                                                C.byref(out)), ctx.handle)
    del keep_b, keep_k
    return Env(out, ctx)


def _info_dict(code, info):
    return {"status": STATUS[code] if code in STATUS else code, "iterations": info.iterations, "outer": info.outer,
            "applies_fp64": info.applies_fp64, "applies_low": info.applies_low, "rel_residual": info.rel_residual,
            "hylleraas": info.hylleraas, "e2": info.e2, "ms_total": info.ms_total}


class Batch:
    """lcc_batch: independent local problems solved together (merged launches, device-side
    scalars and flags, graph-replayed iterations)."""

    def __init__(self, ctx: Context, envs: list):
        self.ctx = ctx
        self.envs = list(envs)
        arr = (C.c_void_p * len(envs))(*[e.handle for e in envs])
        h = C.c_void_p()
        _check(library().lcc_batch_create(ctx.handle, len(envs), arr, C.byref(h)), ctx.handle)
        self.handle = h

    def close(self):
        if self.handle:
            library().lcc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, bs: list, e0s: list, xs: list, vs: list | None = None, precision: str = "fp32",
              tol: float = 1e-10, max_iter: int = 1000, inner_tol: float = 0.0, max_outer: int = 0):
        n = len(self.envs)
        opts = SolveOpts(PRECISIONS[precision], max_iter, tol, inner_tol, max_outer, 0)
        P = C.c_void_p
        barr = (P * n)(*[_tensor_ptr(b, "fp64", e.n) for b, e in zip(bs, self.envs)])
        xarr = (P * n)(*[_tensor_ptr(x, "fp64", e.n) for x, e in zip(xs, self.envs)])
        varr = None
        if vs is not None:
            varr = (P * n)(*[(_tensor_ptr(v, "fp64", e.n) if v is not None else None) for v, e in zip(vs, self.envs)])
        e0 = (C.c_double * n)(*[float(v) for v in e0s])
        infos = (SolveInfo * n)()
        code = library().lcc_batch_solve(self.handle, C.byref(opts), barr, e0, varr, xarr, infos)
        if code < 0:
            _check(code, self.ctx.handle)
        return STATUS[code], [_info_dict(0, i) for i in infos]


def solve_local_lcc_batched(envs: list, bs: list, e0s: list, xs: list, vs: list | None = None,
                            precision: str = "fp32", tol: float = 1e-10, max_iter: int = 1000,
                            inner_tol: float = 0.0, max_outer: int = 0):
    """One-shot batched solve (lcc_solve_local_lcc_batched): creates a batch of `envs`, solves,
    destroys it.  Returns (most severe status, per-problem info dicts)."""
    n = len(envs)
    opts = SolveOpts(PRECISIONS[precision], max_iter, tol, inner_tol, max_outer, 0)
    P = C.c_void_p
    earr = (P * n)(*[e.handle for e in envs])
    barr = (P * n)(*[_tensor_ptr(b, "fp64", e.n) for b, e in zip(bs, envs)])
    xarr = (P * n)(*[_tensor_ptr(x, "fp64", e.n) for x, e in zip(xs, envs)])
    varr = None
    if vs is not None:
        varr = (P * n)(*[(_tensor_ptr(v, "fp64", e.n) if v is not None else None) for v, e in zip(vs, envs)])
    e0 = (C.c_double * n)(*[float(v) for v in e0s])
    infos = (SolveInfo * n)()
    code = library().lcc_solve_local_lcc_batched(n, earr, C.byref(opts), barr, e0, varr, xarr, infos)
    if code < 0:
        _check(code, envs[0].ctx.handle)
    return STATUS[code], [_info_dict(0, i) for i in infos]


class Sweep:
    """lcc_sweep: two-site sweep in both directions (SVD split, truncation, environment update),
    optionally with a reference MPS for first-order problems."""

    def __init__(self, ctx: Context, ham: Hamiltonian, mps: dict, first_site: int):
        self.ctx = ctx
        desc, keep = _mps_desc(mps)
        h = C.c_void_p()
        _check(library().lcc_sweep_create(ctx.handle, ham.handle, C.byref(desc), first_site, C.byref(h)), ctx.handle)
        del keep
        self.handle = h
        self.ham = ham  # the sweep refers to the Hamiltonian's MPO
        self.n_sites = mps["n_sites"]

    def close(self):
        if self.handle:
            library().lcc_sweep_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def env(self) -> "Env":
        """The current block's environment (borrowed; valid until the next advance)."""
        h = C.c_void_p()
        _check(library().lcc_sweep_env(self.handle, C.byref(h)), self.ctx.handle)
        return Env(h, self.ctx)

    def guess(self, x):
        _check(library().lcc_sweep_guess(self.handle, C.c_void_p(x.data_ptr())), self.ctx.handle)

    @staticmethod
    def _info(info) -> dict:
        return {"site": info.site, "kept": info.kept, "n_singular": info.n_singular,
                "discarded_weight": info.discarded_weight, "largest_discarded": info.largest_discarded,
                "ms_svd": info.ms_svd, "ms_env": info.ms_env, "ms_guess": info.ms_guess, "ms_total": info.ms_total}

    def advance(self, x, m_max: int) -> dict:
        info = SweepInfo()
        _check(library().lcc_sweep_advance(self.handle, C.c_void_p(x.data_ptr()), int(m_max), C.byref(info)),
               self.ctx.handle)
        return self._info(info)

    def retreat(self, x, m_max: int) -> dict:
        info = SweepInfo()
        _check(library().lcc_sweep_retreat(self.handle, C.c_void_p(x.data_ptr()), int(m_max), C.byref(info)),
               self.ctx.handle)
        return self._info(info)

    def position(self) -> int:
        site = C.c_int32(0)
        _check(library().lcc_sweep_position(self.handle, C.byref(site)), self.ctx.handle)
        return site.value

    def attach_reference(self, op: Hamiltonian, u: "Hamiltonian | None", ref: dict):
        desc, keep = _mps_desc(ref)
        _check(library().lcc_sweep_attach_reference(self.handle, op.handle, u.handle if u is not None else None,
                                                    C.byref(desc)), self.ctx.handle)
        del keep
        self.refs = (op, u)  # the sweep refers to their MPOs

    def first_order_rhs(self, c: float, b, v) -> float:
        """b = -(P^T O Phi0 - c P^T Phi0), v = P^T Phi0 / |P^T Phi0|; returns |P^T Phi0|."""
        n = C.c_double(0.0)
        _check(library().lcc_sweep_first_order_rhs(self.handle, float(c), C.c_void_p(b.data_ptr()),
                                                   C.c_void_p(v.data_ptr()), C.byref(n)), self.ctx.handle)
        return n.value

    def split_block(self, x, m_max: int) -> dict:
        info = SweepInfo()
        _check(library().lcc_sweep_split_block(self.handle, C.c_void_p(x.data_ptr()), int(m_max), C.byref(info)),
               self.ctx.handle)
        return self._info(info)

    def bond(self, j: int) -> list:
        lib = library()
        n = C.c_int32(0)
        _check(lib.lcc_sweep_bond(self.handle, j, C.byref(n), None), self.ctx.handle)
        arr = (Sector * max(n.value, 1))()
        _check(lib.lcc_sweep_bond(self.handle, j, C.byref(n), arr), self.ctx.handle)
        return [(arr[i].n, arr[i].two_sz, arr[i].dim) for i in range(n.value)]

    def site_tensor(self, j: int) -> list:
        """Blocks [(left sector, s, right sector, array)] of site j (copied to the host)."""
        lib = library()
        nb, ne = C.c_int32(0), C.c_int64(0)
        _check(lib.lcc_sweep_site_tensor(self.handle, j, C.byref(nb), C.byref(ne), None, None), self.ctx.handle)
        blocks = (SiteBlock * max(nb.value, 1))()
        data = np.zeros(max(ne.value, 1))
        _check(lib.lcc_sweep_site_tensor(self.handle, j, C.byref(nb), C.byref(ne), blocks, _dptr(data)),
               self.ctx.handle)
        out = []
        for i in range(nb.value):
            b = blocks[i]
            a = data[b.offset:b.offset + b.rows * b.cols].reshape(b.rows, b.cols).copy()
            out.append((b.left, b.s, b.right, a))
        return out

    def export_mps(self, x, m_max: int, n_elec: int, two_sz: int) -> dict:
        """The sweep's MPS with the block tensor x split in place, as an MPS dict canonical
        around the current block."""
        self.split_block(x, m_max)
        K = self.n_sites
        return {"n_sites": K, "n_elec": n_elec, "two_sz": two_sz, "center": self.position(),
                "bonds": [self.bond(j) for j in range(K + 1)],
                "sites": [self.site_tensor(j) for j in range(K)]}

    def u_expectation(self, x) -> tuple:
        """(x^T U_eff x, x^T x) of the block tensor x."""
        a, b = C.c_double(0.0), C.c_double(0.0)
        _check(library().lcc_sweep_u_expectation(self.handle, C.c_void_p(x.data_ptr()), C.byref(a), C.byref(b)),
               self.ctx.handle)
        return a.value, b.value

    def singular_values(self) -> np.ndarray:
        lib = library()
        n = C.c_int32(0)
        _check(lib.lcc_sweep_singular_values(self.handle, C.byref(n), None))
        out = np.zeros(n.value)
        _check(lib.lcc_sweep_singular_values(self.handle, C.byref(n), _dptr(out)))
        return out



def mps_expectation(ctx: Context, ham: Hamiltonian, mps: dict, site: int | None = None) -> float:
    """lcc_mps_expectation: <Phi|H|Phi> of an MPS canonical around the block (site, site + 1)."""
    if site is None:
        site = mps["center"]
    desc, keep = _mps_desc(mps)
    out = C.c_double(0.0)
    _check(library().lcc_mps_expectation(ctx.handle, ham.handle, C.byref(desc), int(site), C.byref(out)), ctx.handle)
    del keep
    return out.value


def first_order_sweeps(ctx: Context, h0: Hamiltonian, op: Hamiltonian, psi1: dict, psi0: dict, e0: float, c: float,
                       m_max: int, sweeps: int = 2, u: Hamiltonian | None = None, e1: float = 0.0,
                       precision: str = "fp64", tol: float = 1e-10, max_iter: int = 2000) -> dict:
    """First-order MPS-LCC: Phi1 (initial MPS psi1, canonical around its first block) is optimised
    by sweeps of two-site Hylleraas minimisations, (P^T H0 P - E0) x = -P^T Q O Phi0 with x
    orthogonal to P^T Phi0 at every block (lcc_sweep_first_order_rhs, lcc_solve_local_lcc), the
    solved tensor split and truncated to m_max as the sweep moves.  A sweep visits every block of
    the chain once, alternating direction; the first one starts at psi1["center"] and moves right
    (then left).  O = U (op: the part = 2 Hamiltonian, c = E1) or O = H for the projector
    approximation (c = <Phi0|H|Phi0>).  Returns the Hylleraas value of every local solve, the last
    one (E2 = <Phi0|O|Phi1>) and, with u given, E3 = <Phi1|U|Phi1> - E1 <Phi1|Phi1> at the last
    block.  Sequences library calls only; every step runs on the device."""
    import torch
    K = psi1["n_sites"]
    dev = torch.device("cuda", ctx.device if ctx.device >= 0 else 0)
    sw = Sweep(ctx, h0, psi1, psi1["center"])
    try:
        sw.attach_reference(op, u, psi0)
        values, infos = [], []
        direction = 1 if sw.position() < K - 2 else -1
        x = None
        for s in range(sweeps):
            while True:
                env = sw.env()
                b = torch.empty(env.n, dtype=torch.float64, device=dev)
                v = torch.empty_like(b)
                nv = sw.first_order_rhs(c, b, v)
                x = torch.empty_like(b)
                sw.guess(x)
                # the block's basis need not hold Phi0 (it follows Phi1): below 1e-8 the overlap
                # is rounding noise and its direction meaningless, and the constraint is void
                info = env.solve_local_lcc(b, e0, x, v=v if nv > 1e-8 else None, precision=precision, tol=tol,
                                           max_iter=max_iter, inner_tol=1e-4 if precision != "fp64" else 0.0,
                                           max_outer=200)
                if info["status"] not in ("LCC_OK",):
                    raise LccError(-9, f"local solve at site {sw.position()}: {info['status']}")
                values.append(info["hylleraas"])
                infos.append({"site": sw.position(), "sweep": s, "iterations": info["iterations"],
                              "overlap": nv})
                at_end = sw.position() == (K - 2 if direction > 0 else 0)
                if at_end:
                    break
                (sw.advance if direction > 0 else sw.retreat)(x, m_max)
            if s + 1 < sweeps:
                direction = -direction
                (sw.advance if direction > 0 else sw.retreat)(x, m_max)
        out = {"hylleraas": values, "blocks": infos, "e2": values[-1]}
        if u is not None:
            xux, xx = sw.u_expectation(x)
            out["e3"] = xux - e1 * xx
            out["norm2"] = xx
        return out
    finally:
        sw.close()


def dmrg_sweeps(ctx: Context, ham: Hamiltonian, mps: dict, m_max: int, sweeps: int = 2, steps: int = 40,
                tol: float = 1e-10, max_restarts: int = 50) -> dict:
    """Two-site DMRG on the device: at every block the lowest eigenpair of H_eff (restarted
    Lanczos, lcc_lowest_eigenpair, started from the sweep's guess), then the split and move
    (lcc_sweep_advance / _retreat); a sweep visits every block once, alternating direction from
    mps["center"].  Returns the Ritz value of every block and the final MPS (read out with
    lcc_sweep_split_block at the last block).  Sequences library calls only."""
    import torch
    K = mps["n_sites"]
    dev = torch.device("cuda", ctx.device if ctx.device >= 0 else 0)
    sw = Sweep(ctx, ham, mps, mps["center"])
    try:
        energies = []
        direction = 1 if sw.position() < K - 2 else -1
        x = None
        for s in range(sweeps):
            while True:
                env = sw.env()
                x = torch.empty(env.n, dtype=torch.float64, device=dev)
                sw.guess(x)
                info = env.lowest_eigenpair(x, steps=steps, max_restarts=max_restarts, tol=tol, seed=s + 1)
                energies.append(info["theta"])
                if sw.position() == (K - 2 if direction > 0 else 0):
                    break
                (sw.advance if direction > 0 else sw.retreat)(x, m_max)
            if s + 1 < sweeps:
                direction = -direction
                (sw.advance if direction > 0 else sw.retreat)(x, m_max)
        out_mps = sw.export_mps(x, m_max, mps["n_elec"], mps["two_sz"])
        return {"energies": energies, "energy": energies[-1], "mps": out_mps}
    finally:
        sw.close()
