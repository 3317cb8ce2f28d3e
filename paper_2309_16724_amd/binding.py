"""ctypes binding of the C ABI declared in include/dmrg.h.

Argument marshalling only: every step of H.psi and Davidson runs inside the
shared library.  Device memory and streams come from PyTorch (tensors are
passed by data pointer).  Loading fails loudly when the library is missing.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBNAME = "libdmrg_hpsi.so"

c_i32, c_i64, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p

DMRG_FP64 = 0
DMRG_SPLIT_BF16 = 1
DMRG_PLAN_GRAPH = 1
DMRG_PLAN_XCD = 2
DMRG_PLAN_AUTOTUNE = 4
DMRG_RENORM_ALL_PAIRS = 1
DMRG_RENORM_RIGHT = 2


class Sector(ctypes.Structure):
    _fields_ = [("n", c_i32), ("two_s", c_i32), ("dim", c_i32)]


class OpRec(ctypes.Structure):
    _fields_ = [("fam", c_i32), ("row_sec", c_i32), ("col_sec", c_i32), ("npos", c_i32),
                ("off", c_i64)]


class ProblemT(ctypes.Structure):
    _fields_ = [("n_orb", c_i32), ("n_elec", c_i32), ("two_s", c_i32), ("site_l", c_i32),
                ("h1", c_vp), ("eri", c_vp),
                ("n_lsec", c_i32), ("n_rsec", c_i32), ("lsec", c_vp), ("rsec", c_vp),
                ("n_lrec", c_i64), ("n_rrec", c_i64), ("lrec", c_vp), ("rrec", c_vp),
                ("ldata", c_vp), ("rdata", c_vp), ("ldata_len", c_i64), ("rdata_len", c_i64)]


class PlanOpts(ctypes.Structure):
    _fields_ = [("precision", c_i32), ("n_slices", c_i32), ("workspace_bytes", c_i64),
                ("flags", c_i32), ("kpart", c_i32), ("tile_policy", c_i32), ("macro_min", c_i32),
                ("wide_min", c_i32), ("pad_opts", c_i32), ("alloc_fn", c_vp), ("free_fn", c_vp), ("alloc_ctx", c_vp), ("tune_cache", ctypes.c_char_p)]


# device allocator callbacks of dmrg_plan_opts_t
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class DavOpts(ctypes.Structure):
    _fields_ = [("tol", c_dbl), ("max_iter", c_i32), ("m_max", c_i32), ("precond", c_i32),
                ("verbose", c_i32), ("floor", c_dbl), ("mlp", c_vp), ("mlp_patience", c_i32),
                ("pad", c_i32)]


DMRG_PRECOND_DIAG = 0
DMRG_PRECOND_MLP = 1
DMRG_MLP_IN = 2


class TrainOpts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("batch", c_i32), ("steps", c_i32),
                ("seed", ctypes.c_uint64)]


class DavStats(ctypes.Structure):
    _fields_ = [("iters", c_i32), ("n_hpsi", c_i32), ("converged", c_i32), ("fallbacks", c_i32),
                ("residual", c_dbl), ("energy", c_dbl), ("t_total_s", c_dbl), ("t_hpsi_s", c_dbl),
                ("switched", c_i32), ("pad", c_i32), ("sigma", c_dbl)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PlanStats(ctypes.Structure):
    _fields_ = [("psi_len", c_i64), ("n_blocks", c_i64), ("n_rows", c_i64), ("n_tasks", c_i64),
                ("n_stage1", c_i64), ("n_segments", c_i64), ("flops", c_dbl),
                ("stage1_flops", c_dbl), ("stage2_flops", c_dbl), ("workspace_bytes", c_i64),
                ("n_chunks", c_i32), ("kpart", c_i32), ("tile_policy", c_i32), ("xcd", c_i32),
                ("tuned", c_i32), ("launches", c_i32), ("workspace_cap", c_i64), ("tune_ms", c_dbl),
                ("tasks_ms", c_dbl), ("plan_ms", c_dbl), ("macro_min", c_i32), ("wide_min", c_i32),
                ("device_bytes", c_i64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class RKeep(ctypes.Structure):
    _fields_ = [("n", c_i32), ("two_s", c_i32), ("kept", c_i32), ("pad", c_i32), ("u_off", c_i64)]


class RComp(ctypes.Structure):
    _fields_ = [("sec", c_i32), ("l_sec", c_i32), ("site", c_i32), ("row0", c_i32), ("dim", c_i32),
                ("pad", c_i32)]


class RenormStats(ctypes.Structure):
    _fields_ = [("n_terms", c_i64), ("n_products1", c_i64), ("n_products2", c_i64), ("n_tiles1", c_i64),
                ("n_tiles2", c_i64), ("work_elems", c_i64), ("out_elems", c_i64), ("n_records", c_i64), ("flops1", c_dbl),
                ("flops2", c_dbl), ("build_ms", c_dbl)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BlockT(ctypes.Structure):
    _fields_ = [("n_sec", c_i32), ("pad", c_i32), ("sec", c_vp), ("n_rec", c_i64), ("rec", c_vp), ("data", c_vp),
                ("data_len", c_i64)]


class SweepStep(ctypes.Structure):
    _fields_ = [("bond", c_i32), ("kept", c_i32), ("energy", c_dbl), ("kept_weight", c_dbl), ("iters", c_i32),
                ("pad", c_i32)]


_lib = None


def lib_path():
    return os.path.join(HERE, LIBNAME)


def load(path=None):
    """Load the shared library (raises if it was not built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or lib_path()
    if not os.path.exists(p):
        raise RuntimeError("HIP library %s not built; run python -m paper_2309_16724_amd.build" % p)
    L = ctypes.CDLL(p)
    L.dmrg_last_error.restype = ctypes.c_char_p
    for name in ("dmrg_wigner_6j", "dmrg_wigner_9j", "dmrg_ctilde"):
        getattr(L, name).restype = c_dbl
    L.dmrg_wigner_6j.argtypes = [ctypes.c_int] * 6
    L.dmrg_wigner_9j.argtypes = [ctypes.c_int] * 9
    L.dmrg_ctilde.argtypes = [ctypes.c_int] * 9
    L.dmrg_debug_jacobi.argtypes = [c_i32, c_vp, c_vp, c_vp]
    L.dmrg_debug_host_apply.argtypes = [ctypes.POINTER(ProblemT), c_vp, c_vp,
                                        ctypes.POINTER(PlanStats)]
    if hasattr(L, "dmrg_build_tasks"):
        L.dmrg_build_tasks.argtypes = [ctypes.POINTER(ProblemT), c_i32, ctypes.POINTER(PlanOpts),
                                       c_vp, ctypes.POINTER(c_vp)]
        L.dmrg_psi_layout.argtypes = [c_vp, c_i32, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]
        L.dmrg_apply_H.argtypes = [c_vp, c_vp, c_vp, c_vp]
        L.dmrg_apply_H_static.argtypes = [c_vp, c_vp, c_vp, c_vp]
        L.dmrg_diag_H.argtypes = [c_vp, c_vp, c_vp]
        L.dmrg_plan_stats.argtypes = [c_vp, ctypes.POINTER(PlanStats)]
        L.dmrg_plan_free.argtypes = [c_vp]
        L.dmrg_plan_free.restype = None
        L.dmrg_davidson.argtypes = [c_vp, c_vp, ctypes.POINTER(c_dbl), ctypes.POINTER(DavOpts),
                                    ctypes.POINTER(DavStats), c_vp]
        L.dmrg_set_profiling.argtypes = [c_vp, c_i32]
        L.dmrg_get_profile.argtypes = [c_vp, c_i32, ctypes.POINTER(c_i64), ctypes.POINTER(c_dbl),
                                       ctypes.POINTER(c_dbl)]
        L.dmrg_debug_plan_host_apply.argtypes = [ctypes.POINTER(ProblemT), c_vp, c_vp,
                                                 ctypes.POINTER(PlanOpts), ctypes.POINTER(PlanStats)]
        L.dmrg_debug_plan_tiles.argtypes = [ctypes.POINTER(ProblemT), ctypes.POINTER(PlanOpts), c_i32, c_vp, c_i64]
        L.dmrg_debug_plan_tiles.restype = c_i64
        c_f = ctypes.c_float
        L.dmrg_mlp_create.argtypes = [c_i32, ctypes.c_uint64, ctypes.POINTER(c_vp)]
        L.dmrg_mlp_num_params.argtypes = [c_vp]
        L.dmrg_mlp_step.argtypes = [c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_dbl, c_vp, c_vp]
        L.dmrg_mlp_num_params.restype = c_i64
        L.dmrg_mlp_set_params.argtypes = [c_vp, c_vp, c_i64]
        L.dmrg_mlp_get_params.argtypes = [c_vp, c_vp, c_i64]
        L.dmrg_mlp_forward.argtypes = [c_vp, c_vp, c_i64, c_vp, c_vp]
        L.dmrg_mlp_loss_grad.argtypes = [c_vp, c_vp, c_vp, c_vp, c_i64, ctypes.POINTER(c_dbl), c_vp,
                                         c_vp]
        L.dmrg_mlp_adam_step.argtypes = [c_vp, c_vp, c_f, c_f, c_f, c_f, c_vp]
        L.dmrg_mlp_train.argtypes = [c_vp, c_vp, c_vp, c_vp, c_i64, ctypes.POINTER(TrainOpts), c_vp,
                                     c_vp]
        L.dmrg_mlp_collect.argtypes = [c_vp, c_vp, ctypes.POINTER(DavOpts), c_i64, c_vp, c_vp, c_vp,
                                       ctypes.POINTER(c_i64), ctypes.POINTER(c_i32), c_vp]
        L.dmrg_mlp_free.argtypes = [c_vp]
        L.dmrg_mlp_free.restype = None
    if hasattr(L, "dmrg_renorm_create"):
        L.dmrg_renorm_product.argtypes = [ctypes.POINTER(ProblemT), c_i32, c_vp, c_i32, ctypes.POINTER(c_i32),
                                          c_vp, c_i32, ctypes.POINTER(c_i32)]
        L.dmrg_renorm_create.argtypes = [ctypes.POINTER(ProblemT), c_vp, c_i32, c_i32, c_i32, c_i64,
                                         ctypes.POINTER(c_vp)]
        L.dmrg_renorm_records.argtypes = [c_vp, c_vp, c_i64, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]
        L.dmrg_renorm_apply.argtypes = [c_vp, c_vp, c_vp, c_vp]
        L.dmrg_renorm_stats.argtypes = [c_vp, ctypes.POINTER(RenormStats)]
        L.dmrg_renorm_set_profiling.argtypes = [c_vp, c_i32]
        L.dmrg_debug_truncate_rho_host.argtypes = [ctypes.POINTER(ProblemT), c_i32, c_vp, c_vp, c_i64,
                                                   ctypes.POINTER(c_i64)]
        L.dmrg_sweep_left_to_right.argtypes = [c_i32, c_i32, c_i32, c_vp, c_vp, c_i32, ctypes.POINTER(BlockT),
                                               ctypes.POINTER(BlockT), c_i32, c_vp, c_vp, ctypes.c_uint64, c_vp,
                                               c_vp, c_vp]
        L.dmrg_block_release.argtypes = [ctypes.POINTER(BlockT)]
        L.dmrg_block_release.restype = None
        L.dmrg_sweep_right_to_left.argtypes = L.dmrg_sweep_left_to_right.argtypes
        L.dmrg_truncate.argtypes = [ctypes.POINTER(ProblemT), c_i32, c_vp, c_i32, c_dbl, c_vp, c_i32, ctypes.POINTER(c_i32),
                                    c_vp, c_i64, ctypes.POINTER(c_i64), c_vp, c_vp]
        L.dmrg_renorm_get_profile.argtypes = [c_vp, c_i32, ctypes.POINTER(c_i64), ctypes.POINTER(c_dbl),
                                              ctypes.POINTER(c_dbl)]
        L.dmrg_renorm_free.argtypes = [c_vp]
        L.dmrg_renorm_free.restype = None
        L.dmrg_debug_renorm_host.argtypes = [ctypes.POINTER(ProblemT), c_vp, c_i32, c_i32, c_i32, c_vp, c_i64,
                                             c_vp, c_i64, c_vp, c_i64, ctypes.POINTER(RenormStats)]
    if path is None:
        _lib = L
    return L


def check(rc, L=None):
    if rc != 0:
        L = L or load()
        raise RuntimeError("dmrg error %d: %s" % (rc, L.dmrg_last_error().decode()))


class ProblemArgs:
    """Keeps host arrays alive and exposes the C struct of one problem.

    ``ldata``/``rdata`` are integer addresses of the operator data (device
    pointers for the GPU path, host pointers for the debug host evaluation).
    """

    def __init__(self, prob, ldata_ptr, rdata_ptr):
        self.h1 = np.ascontiguousarray(prob.h, dtype=np.float64)
        self.eri = np.ascontiguousarray(prob.eri, dtype=np.float64)
        self.lsec = (Sector * len(prob.left.sectors))(*[Sector(*s) for s in prob.left.sectors])
        self.rsec = (Sector * len(prob.right.sectors))(*[Sector(*s) for s in prob.right.sectors])
        lr, rr = prob.left.records, prob.right.records
        self.lrec = (OpRec * max(1, len(lr)))(*[OpRec(f, r, c, n, o) for (f, r, c, o, n) in lr])
        self.rrec = (OpRec * max(1, len(rr)))(*[OpRec(f, r, c, n, o) for (f, r, c, o, n) in rr])
        self.s = ProblemT(prob.n_orb, prob.n_elec, prob.two_s, prob.p,
                          self.h1.ctypes.data, self.eri.ctypes.data,
                          len(prob.left.sectors), len(prob.right.sectors),
                          ctypes.addressof(self.lsec), ctypes.addressof(self.rsec),
                          len(lr), len(rr), ctypes.addressof(self.lrec), ctypes.addressof(self.rrec),
                          ldata_ptr, rdata_ptr, prob.left.data.size, prob.right.data.size)


def debug_plan_host_apply(prob, psi, workspace_bytes=0, lib=None, precision=0, n_slices=0, kpart=0,
                          tile_policy=0, macro_min=0, wide_min=0):
    """Test-only: run the device plan's tile lists on the CPU (no GPU).

    ``psi=None`` only builds the plan and returns its statistics."""
    L = lib or load()
    ld = np.ascontiguousarray(prob.left.data)
    rd = np.ascontiguousarray(prob.right.data)
    args = ProblemArgs(prob, ld.ctypes.data, rd.ctypes.data)
    st = PlanStats()
    opts = PlanOpts(precision, n_slices, workspace_bytes, 0, kpart, tile_policy, macro_min, wide_min, 0,
                    None, None, None, None)
    if psi is None:
        check(L.dmrg_debug_plan_host_apply(ctypes.byref(args.s), None, None, ctypes.byref(opts),
                                           ctypes.byref(st)), L)
        return None, st.as_dict()
    x = np.ascontiguousarray(psi, dtype=np.float64)
    y = np.zeros_like(x)
    check(L.dmrg_debug_plan_host_apply(ctypes.byref(args.s), x.ctypes.data, y.ctypes.data,
                                       ctypes.byref(opts), ctypes.byref(st)), L)
    return y, st.as_dict()


def debug_plan_tiles(prob, stage, lib=None, precision=0, n_slices=0, kpart=0, tile_policy=0, macro_min=0,
                     wide_min=0):
    """Test-only: the tiles of one stage of the plan for one problem, an
    array of rows (rows, columns, segments, summed K, output rows, output
    columns, kind) -- see dmrg_debug_plan_tiles."""
    L = lib or load()
    ld = np.ascontiguousarray(prob.left.data)
    rd = np.ascontiguousarray(prob.right.data)
    args = ProblemArgs(prob, ld.ctypes.data, rd.ctypes.data)
    opts = PlanOpts(precision, n_slices, 0, 0, kpart, tile_policy, macro_min, wide_min, 0, None, None, None, None)
    n = L.dmrg_debug_plan_tiles(ctypes.byref(args.s), ctypes.byref(opts), stage, None, 0)
    if n < 0:
        check(int(n), L)
    out = np.zeros((max(n, 1), 7), dtype=np.int64)
    L.dmrg_debug_plan_tiles(ctypes.byref(args.s), ctypes.byref(opts), stage, out.ctypes.data, n)
    return out[:n]


def debug_jacobi(A, lib=None, sweeps=False):
    """Test-only: eigenvalues (ascending) and eigenvectors (columns) of a
    symmetric m x m matrix by the Davidson solver's host Jacobi routine
    (and the number of sweeps it ran with sweeps=True)."""
    L = lib or load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    m = A.shape[0]
    w = np.zeros(m)
    Z = np.zeros((m, m))
    n = L.dmrg_debug_jacobi(m, A.ctypes.data, w.ctypes.data, Z.ctypes.data)
    check(min(n, 0), L)
    return (w, Z, n) if sweeps else (w, Z)


def debug_host_apply(prob, psi, lib=None):
    """Test-only: evaluate the host task list on the CPU (no GPU)."""
    L = lib or load()
    ld = np.ascontiguousarray(prob.left.data)
    rd = np.ascontiguousarray(prob.right.data)
    args = ProblemArgs(prob, ld.ctypes.data, rd.ctypes.data)
    x = np.ascontiguousarray(psi, dtype=np.float64)
    y = np.zeros_like(x)
    st = PlanStats()
    check(L.dmrg_debug_host_apply(ctypes.byref(args.s), x.ctypes.data, y.ctypes.data,
                                  ctypes.byref(st)), L)
    return y, st


def renorm_product(prob, lib=None, right=False):
    """Product basis of the left block x site (right: site x right block):
    [(n, 2S, rows)] and components [(sector, block sector, site multiplet,
    row0, dim)] (dmrg_renorm_product)."""
    L = lib or load()
    args = ProblemArgs(prob, 0, 0)
    fl = DMRG_RENORM_RIGHT if right else 0
    ns, nc = c_i32(), c_i32()
    check(L.dmrg_renorm_product(ctypes.byref(args.s), fl, None, 0, ctypes.byref(ns), None, 0, ctypes.byref(nc)), L)
    sec = (Sector * max(1, ns.value))()
    comp = (RComp * max(1, nc.value))()
    check(L.dmrg_renorm_product(ctypes.byref(args.s), fl, ctypes.addressof(sec), ns.value, ctypes.byref(ns),
                                ctypes.addressof(comp), nc.value, ctypes.byref(nc)), L)
    return ([(s.n, s.two_s, s.dim) for s in sec[:ns.value]],
            [(c.sec, c.l_sec, c.site, c.row0, c.dim) for c in comp[:nc.value]])


def keep_array(keep):
    """keep: [(n, 2S, U)] -> (RKeep array, flat U (column-major per sector), length)."""
    offs, parts, off = [], [], 0
    for (n, S, U) in keep:
        U = np.asarray(U, dtype=np.float64)
        offs.append(RKeep(n, S, U.shape[1], 0, off))
        parts.append(np.asfortranarray(U).reshape(-1, order="F"))
        off += U.size
    arr = (RKeep * len(offs))(*offs)
    flat = np.concatenate(parts) if parts else np.zeros(1)
    return arr, flat, off


def records_block(prob, keep, recs, data, right=False):
    """Output of a renormalization as BlockData (role L at bond p + 1, or
    role R at bond p - 1 for the right block)."""
    from .synth.problem import BlockData
    secs = [(n, S, np.asarray(U).shape[1]) for (n, S, U) in keep]
    if right:
        blk = BlockData("R", prob.n_orb, prob.p - 1, secs)
    else:
        blk = BlockData("L", prob.n_orb, prob.p + 1, secs, all_pairs=getattr(prob.left, "all_pairs", False))
    blk.records = [(r.fam, r.row_sec, r.col_sec, r.off, r.npos) for r in recs]
    blk.data = np.asarray(data, dtype=np.float64)
    return blk


def debug_renorm_host(prob, keep, fam_mask=0, lib=None, execute=True, right=False):
    """Test-only: the renormalization lists executed on the CPU (no GPU).
    Returns (BlockData of the new block or None, statistics)."""
    L = lib or load()
    ld = np.ascontiguousarray(prob.left.data)
    rd = np.ascontiguousarray(prob.right.data)
    args = ProblemArgs(prob, ld.ctypes.data, rd.ctypes.data)
    karr, u, ulen = keep_array(keep)
    st = RenormStats()
    if right:
        flags = DMRG_RENORM_RIGHT
    else:
        flags = DMRG_RENORM_ALL_PAIRS if getattr(prob.left, "all_pairs", False) else 0
    check(L.dmrg_debug_renorm_host(ctypes.byref(args.s), ctypes.addressof(karr), len(keep), fam_mask, flags,
                                   None, ulen, None, 0, None, 0, ctypes.byref(st)), L)
    if not execute:
        return None, st.as_dict()
    out = np.zeros(max(1, st.out_elems))
    recs = (OpRec * max(1, st.n_records))()
    check(L.dmrg_debug_renorm_host(ctypes.byref(args.s), ctypes.addressof(karr), len(keep), fam_mask, flags,
                                   u.ctypes.data, ulen, out.ctypes.data, out.size, ctypes.addressof(recs),
                                   st.n_records, ctypes.byref(st)), L)
    return records_block(prob, keep, recs[:st.n_records], out[:st.out_elems], right), st.as_dict()


def debug_truncate_rho_host(prob, psi, right=False, lib=None):
    """Test-only: dmrg_debug_truncate_rho_host -> {(n, 2S): rho} in product order."""
    L = lib or load()
    args = ProblemArgs(prob, 0, 0)
    fl = DMRG_RENORM_RIGHT if right else 0
    n = c_i64()
    check(L.dmrg_debug_truncate_rho_host(ctypes.byref(args.s), fl, None, None, 0, ctypes.byref(n)), L)
    x = np.ascontiguousarray(psi, dtype=np.float64)
    rho = np.zeros(max(1, n.value))
    check(L.dmrg_debug_truncate_rho_host(ctypes.byref(args.s), fl, x.ctypes.data, rho.ctypes.data, rho.size,
                                         ctypes.byref(n)), L)
    secs, _ = renorm_product(prob, L, right=right)
    out, off = {}, 0
    for (sn, s2, rows) in secs:
        out[(sn, s2)] = rho[off:off + rows * rows].reshape(rows, rows).T.copy()
        off += rows * rows
    return out
