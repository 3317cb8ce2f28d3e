"""Python handle on a device plan (argument marshalling over the C ABI).

Operator data are copied to the GPU once; psi/hpsi are torch CUDA tensors
passed by pointer.  Nothing here computes: H.psi, diag(H) and Davidson run
in the HIP library.  If the library is missing, construction raises.
"""
import ctypes

import numpy as np

from . import binding as B


def _torch():
    import torch
    return torch


class TorchAllocator:
    """Device-memory callbacks for dmrg_plan_opts_t that take the plan's
    memory from PyTorch's caching allocator on a given stream (counting
    calls, bytes and live blocks)."""

    def __init__(self, device, stream=None):
        torch = _torch()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.calls = self.frees = 0
        self.bytes = 0
        self.live = {}

        def _alloc(n, ctx):
            try:
                p = torch.cuda.caching_allocator_alloc(int(n), self.device.index or 0, self.stream)
            except Exception:
                return None
            self.calls += 1
            self.bytes += int(n)
            self.live[int(p)] = int(n)
            return int(p)

        def _free(p, ctx):
            if p:
                self.live.pop(int(p), None)
                self.frees += 1
                torch.cuda.caching_allocator_delete(int(p))

        self.alloc_fn = B.ALLOC_FN(_alloc)
        self.free_fn = B.FREE_FN(_free)


class Plan:
    def __init__(self, problems, precision=B.DMRG_FP64, n_slices=0, workspace_bytes=0,
                 device="cuda:0", flags=0, kpart=0, tile_policy=0, macro_min=0, allocator=None,
                 tune_cache=None, wide_min=0):
        """allocator: None (the library uses hipMalloc), "torch" (PyTorch's
        caching allocator on the current stream) or a TorchAllocator;
        tune_cache: file of autotuned settings (with DMRG_PLAN_AUTOTUNE)."""
        torch = _torch()
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        self.lib = B.load()
        if not hasattr(self.lib, "dmrg_build_tasks"):
            raise RuntimeError("library has no GPU entry points")
        self.device = torch.device(device)
        self.problems = problems
        self._keep = []
        structs = []
        for pr in problems:
            ld = torch.from_numpy(np.ascontiguousarray(pr.left.data)).to(self.device)
            rd = torch.from_numpy(np.ascontiguousarray(pr.right.data)).to(self.device)
            if ld.numel() == 0:
                ld = torch.zeros(1, dtype=torch.float64, device=self.device)
            if rd.numel() == 0:
                rd = torch.zeros(1, dtype=torch.float64, device=self.device)
            args = B.ProblemArgs(pr, ld.data_ptr(), rd.data_ptr())
            self._keep += [ld, rd, args]
            structs.append(args.s)
        arr = (B.ProblemT * len(structs))(*structs)
        self._keep.append(arr)
        if allocator == "torch":
            allocator = TorchAllocator(device)
        self.allocator = allocator
        fa = ctypes.cast(allocator.alloc_fn, ctypes.c_void_p) if allocator is not None else None
        ff = ctypes.cast(allocator.free_fn, ctypes.c_void_p) if allocator is not None else None
        tc = None if tune_cache is None else str(tune_cache).encode()
        self._keep.append(tc)
        opts = B.PlanOpts(precision, n_slices, workspace_bytes, flags, kpart, tile_policy, macro_min,
                          wide_min, 0, fa, ff, None, tc)
        h = ctypes.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        torch.cuda.synchronize(self.device)
        B.check(self.lib.dmrg_build_tasks(arr, len(structs), ctypes.byref(opts),
                                          ctypes.c_void_p(stream), ctypes.byref(h)), self.lib)
        self.handle = h
        st = self.stats()
        self.size = int(st["psi_len"])

    def stats(self):
        st = B.PlanStats()
        B.check(self.lib.dmrg_plan_stats(self.handle, ctypes.byref(st)), self.lib)
        return st.as_dict()

    def layout(self, k):
        off, ln = ctypes.c_int64(), ctypes.c_int64()
        B.check(self.lib.dmrg_psi_layout(self.handle, k, ctypes.byref(off), ctypes.byref(ln)), self.lib)
        return off.value, ln.value

    def _stream(self, stream):
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(s.cuda_stream)

    def apply(self, psi, out=None, stream=None):
        torch = _torch()
        assert psi.dtype == torch.float64 and psi.is_cuda and psi.numel() == self.size
        psi = psi.contiguous()
        if out is None:
            out = torch.empty_like(psi)
        B.check(self.lib.dmrg_apply_H(self.handle, ctypes.c_void_p(psi.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), self._stream(stream)), self.lib)
        return out

    def apply_static(self, psi, out, stream=None):
        """H.psi through dmrg_apply_H_static (the library's static scratch
        array, no device allocation in the call); out: preallocated tensor."""
        torch = _torch()
        assert psi.dtype == torch.float64 and psi.is_cuda and psi.numel() == self.size
        assert out.dtype == torch.float64 and out.is_cuda and out.numel() == self.size
        B.check(self.lib.dmrg_apply_H_static(self.handle, ctypes.c_void_p(psi.data_ptr()),
                                             ctypes.c_void_p(out.data_ptr()), self._stream(stream)), self.lib)
        return out

    def diag(self, out=None, stream=None):
        torch = _torch()
        if out is None:
            out = torch.empty(self.size, dtype=torch.float64, device=self.device)
        B.check(self.lib.dmrg_diag_H(self.handle, ctypes.c_void_p(out.data_ptr()),
                                     self._stream(stream)), self.lib)
        return out

    def davidson(self, psi0, tol=1e-8, max_iter=1000, m_max=24, floor=1e-2, stream=None,
                 check=True, mlp=None, verbose=0, mlp_patience=0):
        """Lowest eigenpair of every problem by the library's Davidson solver.

        psi0: CUDA float64 tensor (starting vectors, not modified); mlp: a
        precond.MLP for the learned preconditioner, else the diagonal one;
        mlp_patience: iterations without a new smallest residual after which a
        problem's learned steps stop (0: the library default).
        Returns (energy, psi, stats dict): energy is the Ritz value of a
        single-problem plan, else the list of Ritz values, one per problem.
        With check=False a non-converged run returns its best pairs instead of
        raising."""
        torch = _torch()
        assert psi0.dtype == torch.float64 and psi0.is_cuda and psi0.numel() == self.size
        psi = psi0.detach().clone().contiguous()
        ev = (ctypes.c_double * len(self.problems))()
        st = B.DavStats()
        opts = self._dav_opts(tol, max_iter, m_max, floor, mlp, verbose, mlp_patience)
        rc = self.lib.dmrg_davidson(self.handle, ctypes.c_void_p(psi.data_ptr()), ev,
                                    ctypes.byref(opts), ctypes.byref(st), self._stream(stream))
        if rc != 0 and (check or rc != -7):
            B.check(rc, self.lib)
        torch.cuda.synchronize(self.device)
        evs = list(ev)
        return (evs[0] if len(evs) == 1 else evs), psi, st.as_dict()

    @staticmethod
    def _dav_opts(tol, max_iter, m_max, floor, mlp=None, verbose=0, mlp_patience=0):
        if mlp is None:
            return B.DavOpts(tol, max_iter, m_max, B.DMRG_PRECOND_DIAG, verbose, floor, None, mlp_patience, 0)
        return B.DavOpts(tol, max_iter, m_max, B.DMRG_PRECOND_MLP, verbose, floor, mlp.handle, mlp_patience, 0)

    def collect(self, psi0, capacity, tol=1e-8, max_iter=1000, m_max=24, floor=1e-2,
                stream=None):
        """Training rows (x, a, b) of the learned preconditioner from this
        single-problem plan's solve (see dmrg_mlp_collect): CUDA float32
        tensors trimmed to the recorded rows, and the number of iterations."""
        torch = _torch()
        assert psi0.dtype == torch.float64 and psi0.is_cuda and psi0.numel() == self.size
        x = torch.empty((capacity, B.DMRG_MLP_IN), dtype=torch.float32, device=self.device)
        a = torch.empty(capacity, dtype=torch.float32, device=self.device)
        b = torch.empty(capacity, dtype=torch.float32, device=self.device)
        nr, nrec = ctypes.c_int64(), ctypes.c_int32()
        opts = self._dav_opts(tol, max_iter, m_max, floor)
        B.check(self.lib.dmrg_mlp_collect(self.handle, ctypes.c_void_p(psi0.data_ptr()),
                                          ctypes.byref(opts), capacity,
                                          ctypes.c_void_p(x.data_ptr()),
                                          ctypes.c_void_p(a.data_ptr()),
                                          ctypes.c_void_p(b.data_ptr()), ctypes.byref(nr),
                                          ctypes.byref(nrec), self._stream(stream)), self.lib)
        torch.cuda.synchronize(self.device)
        n = nr.value
        return x[:n], a[:n], b[:n], nrec.value

    def set_profiling(self, on=True):
        B.check(self.lib.dmrg_set_profiling(self.handle, 1 if on else 0), self.lib)

    def profile(self, stage):
        """(launches, total ms, total algorithmic flops) of stage 1 or 2 since set_profiling."""
        n, ms, fl = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        B.check(self.lib.dmrg_get_profile(self.handle, stage, ctypes.byref(n), ctypes.byref(ms),
                                          ctypes.byref(fl)), self.lib)
        return n.value, ms.value, fl.value

    def free(self):
        if getattr(self, "handle", None):
            _torch().cuda.synchronize(self.device)
            self.lib.dmrg_plan_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Renorm:
    """Renormalization of a problem's left block through its left site on the
    GPU (dmrg_renorm_*): the families H, C, A0, A1, B0, B1, S (and P, Q for a
    left block that holds them for every outside pair) of the block
    [0, site_l] in the kept basis.  ``keep`` is [(n, 2S, U)] with U a host
    array (rows of that product sector x kept) or ``u`` a device tensor that
    already holds the matrices at the offsets ``keep_array`` would give."""

    def __init__(self, prob, keep, device="cuda:0", fam_mask=0, ldata=None, right=False):
        """right: renormalize the right block through the right site instead
        (``ldata`` then stands for the right block's device data)."""
        torch = _torch()
        self.lib = B.load()
        if not hasattr(self.lib, "dmrg_renorm_create"):
            raise RuntimeError("library has no renormalization entry points")
        self.device = torch.device(device)
        self.prob, self.keep = prob, keep
        self.right = right
        blk = prob.right if right else prob.left
        self.ld = ldata if ldata is not None else \
            torch.from_numpy(np.ascontiguousarray(blk.data)).to(self.device)
        self.args = B.ProblemArgs(prob, 0 if right else self.ld.data_ptr(), self.ld.data_ptr() if right else 0)
        self.karr, flat, self.u_len = B.keep_array(keep)
        self.u = torch.from_numpy(flat).to(self.device)
        h = ctypes.c_void_p()
        if right:
            flags = B.DMRG_RENORM_RIGHT
        else:
            flags = B.DMRG_RENORM_ALL_PAIRS if getattr(prob.left, "all_pairs", False) else 0
        B.check(self.lib.dmrg_renorm_create(ctypes.byref(self.args.s), ctypes.addressof(self.karr), len(keep),
                                            fam_mask, flags, self.u_len, ctypes.byref(h)), self.lib)
        self.handle = h
        n, ln = ctypes.c_int64(), ctypes.c_int64()
        B.check(self.lib.dmrg_renorm_records(self.handle, None, 0, ctypes.byref(n), ctypes.byref(ln)), self.lib)
        self.recs = (B.OpRec * max(1, n.value))()
        B.check(self.lib.dmrg_renorm_records(self.handle, ctypes.addressof(self.recs), n.value, ctypes.byref(n),
                                             ctypes.byref(ln)), self.lib)
        self.n_rec, self.out_len = n.value, ln.value
        self.out = torch.empty(max(1, self.out_len), dtype=torch.float64, device=self.device)

    def stats(self):
        st = B.RenormStats()
        B.check(self.lib.dmrg_renorm_stats(self.handle, ctypes.byref(st)), self.lib)
        return st.as_dict()

    def apply(self, stream=None):
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        B.check(self.lib.dmrg_renorm_apply(self.handle, ctypes.c_void_p(self.u.data_ptr()),
                                           ctypes.c_void_p(self.out.data_ptr()), ctypes.c_void_p(s.cuda_stream)),
                self.lib)
        return self.out

    def set_profiling(self, on=True):
        B.check(self.lib.dmrg_renorm_set_profiling(self.handle, 1 if on else 0), self.lib)

    def profile(self, stage):
        """(launches, total ms, total algorithmic flops) of stage 1 or 2 since set_profiling."""
        n, ms, fl = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        B.check(self.lib.dmrg_renorm_get_profile(self.handle, stage, ctypes.byref(n), ctypes.byref(ms),
                                                 ctypes.byref(fl)), self.lib)
        return n.value, ms.value, fl.value

    def block(self):
        """The new block as host BlockData (after apply)."""
        _torch().cuda.synchronize(self.device)
        return B.records_block(self.prob, self.keep, self.recs[:self.n_rec],
                               self.out[:self.out_len].cpu().numpy(), self.right)

    def free(self):
        if getattr(self, "handle", None):
            _torch().cuda.synchronize(self.device)
            self.lib.dmrg_renorm_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def truncate(prob, psi, max_kept, cutoff=0.0, stream=None, right=False):
    """Kept multiplets of (left block x left site) from the reduced density
    matrix of psi (a device tensor of the problem's reduced coefficients):
    (keep [(n, 2S, kept, u_off)], u device tensor, (kept weight, trace)) --
    dmrg_truncate; ``keep_host`` turns them into the [(n, 2S, U)] that
    Renorm takes."""
    torch = _torch()
    lib = B.load()
    s = stream if stream is not None else torch.cuda.current_stream(psi.device)
    args = B.ProblemArgs(prob, 0, 0)
    nk, ul = ctypes.c_int32(), ctypes.c_int64()
    w = (ctypes.c_double * 2)()
    fl = B.DMRG_RENORM_RIGHT if right else 0
    B.check(lib.dmrg_truncate(ctypes.byref(args.s), fl, ctypes.c_void_p(psi.data_ptr()), max_kept, cutoff, None, 0,
                              ctypes.byref(nk), None, 0, ctypes.byref(ul), w, ctypes.c_void_p(s.cuda_stream)), lib)
    karr = (B.RKeep * max(1, nk.value))()
    u = torch.empty(max(1, ul.value), dtype=torch.float64, device=psi.device)
    B.check(lib.dmrg_truncate(ctypes.byref(args.s), fl, ctypes.c_void_p(psi.data_ptr()), max_kept, cutoff,
                              ctypes.addressof(karr), nk.value, ctypes.byref(nk), ctypes.c_void_p(u.data_ptr()),
                              u.numel(), ctypes.byref(ul), w, ctypes.c_void_p(s.cuda_stream)), lib)
    keep = [(k.n, k.two_s, k.kept, k.u_off) for k in karr[:nk.value]]
    return keep, u, (w[0], w[1])


def keep_host(prob, keep, u, right=False):
    """[(n, 2S, U host array)] from truncate's outputs (rows from the product basis)."""
    secs, _ = B.renorm_product(prob, right=right)
    rows = {(n, s2): r for (n, s2, r) in secs}
    uh = u.cpu().numpy()
    out = []
    for (n, s2, kept, off) in keep:
        r = rows[(n, s2)]
        out.append((n, s2, uh[off:off + r * kept].reshape(kept, r).T.copy()))
    return out


def catalogue_left(blk):
    """The H.psi form of a left block that holds P and Q for every outside
    pair: its P0, P1, Q0, Q1 records cut to the pairs that touch the two
    sites (a selection of positions, no arithmetic)."""
    from .synth.problem import BlockData
    from .synth import catalogue as cat
    if not getattr(blk, "all_pairs", False):
        return blk
    out = BlockData(blk.role, blk.n_orb, blk.p, blk.sectors)
    recs, chunks, off = [], [], 0
    for (f, r, c, o, npos) in blk.records:
        dr, dc = blk.sectors[r][2], blk.sectors[c][2]
        arr = blk.data[o:o + npos * dr * dc].reshape(npos, dr * dc)
        if f in (cat.P0, cat.P1, cat.Q0, cat.Q1):
            full = cat.labels(f, "L", blk.n_orb, blk.p, True)
            arr = arr[[full.index(lab) for lab in cat.labels(f, "L", blk.n_orb, blk.p)]]
        if arr.shape[0] == 0:
            continue
        recs.append((f, r, c, off, arr.shape[0]))
        chunks.append(arr.reshape(-1))
        off += arr.size
    out.records = recs
    out.data = np.concatenate(chunks) if chunks else np.zeros(0)
    return out


def sweep_left_to_right(left, rights, h, eri, n_elec, two_s, D, tol=1e-9, seed=100, device="cuda:0"):
    """One left-to-right two-site sweep through the library's entry points:
    at every bond p from left.p to the last, the two-site problem of the
    left block (P and Q over every outside pair) and rights[p] is solved by
    Davidson (dmrg_davidson), its wavefunction cut to at most D multiplets of
    (left block x site) (dmrg_truncate) and the left block renormalized with
    that basis (dmrg_renorm_*, all-pairs form) into the left block of the
    next bond.  Returns [(bond, energy, kept multiplets, kept weight)]."""
    torch = _torch()
    from .synth.problem import Problem, random_vector
    n_orb = h.shape[0]
    out = []
    for p in range(left.p, n_orb - 1):
        prob = Problem(n_orb, n_elec, two_s, p, h, eri, catalogue_left(left), rights[p])
        plan = Plan(prob, device=device)
        x = random_vector(plan.size, seed + p)
        x0 = torch.from_numpy(x / np.linalg.norm(x)).to(device)
        e, psi, st = plan.davidson(x0, tol=tol)
        plan.free()
        if p == n_orb - 2:
            out.append((p, e, None, None))
            break
        keep, u, (kw, tr) = truncate(prob, psi, D, 1e-14)
        full = Problem(n_orb, n_elec, two_s, p, h, eri, left, rights[p])
        r = Renorm(full, keep_host(full, keep, u), device=device)
        r.apply()
        left = r.block()
        r.free()
        out.append((p, e, sum(k[2] for k in keep), kw / tr))
    return out


def sweep_right_to_left(lefts, right, h, eri, n_elec, two_s, D, tol=1e-9, seed=200, device="cuda:0"):
    """One right-to-left two-site sweep, the mirror of sweep_left_to_right:
    at every bond p from right.p down to 0, the problem of lefts[p] (the
    H.psi form) and the right block is solved by Davidson, cut to at most D
    multiplets of (right site x right block) (dmrg_truncate with the right
    flag) and the right block renormalized with that basis into the right
    block of bond p - 1.  Returns [(bond, energy, kept, kept weight)]."""
    torch = _torch()
    from .synth.problem import Problem, random_vector
    n_orb = h.shape[0]
    out = []
    for p in range(right.p, -1, -1):
        prob = Problem(n_orb, n_elec, two_s, p, h, eri, catalogue_left(lefts[p]), right)
        plan = Plan(prob, device=device)
        x = random_vector(plan.size, seed + p)
        x0 = torch.from_numpy(x / np.linalg.norm(x)).to(device)
        e, psi, st = plan.davidson(x0, tol=tol)
        plan.free()
        if p == 0:
            out.append((p, e, None, None))
            break
        keep, u, (kw, tr) = truncate(prob, psi, D, 1e-14, right=True)
        r = Renorm(prob, keep_host(prob, keep, u, right=True), device=device, right=True)
        r.apply()
        right = r.block()
        r.free()
        out.append((p, e, sum(k[2] for k in keep), kw / tr))
    return out



def sweep_native(blocks, grown, h, eri, n_elec, two_s, D, tol=1e-9, seed=100, device="cuda:0", stream=None,
                 right_to_left=False, keep_blocks=False, precision=B.DMRG_FP64, n_slices=0):
    """A sweep inside the library, every grown block kept on the device.
    Left to right (dmrg_sweep_left_to_right): grown is the all-pairs left
    block of bond grown.p, blocks = {bond: right block}.  Right to left
    (dmrg_sweep_right_to_left): grown is the right block of bond grown.p,
    blocks = {bond: left block}; a block is a BlockData or a BlockT that
    an earlier sweep returned (device data).  Returns [(bond, energy, kept,
    kept weight, iterations)] in sweep order, and with keep_blocks also the
    grown blocks as BlockT (entry i: grown at step i; release_blocks frees
    them).  precision / n_slices: the plans' arithmetic (dmrg_plan_opts_t)."""
    torch = _torch()
    lib = B.load()
    n_orb = h.shape[0]
    keepalive = []

    def block(blk):
        if isinstance(blk, B.BlockT):
            return blk
        sec = (B.Sector * max(1, len(blk.sectors)))(*[B.Sector(*x) for x in blk.sectors])
        rec = (B.OpRec * max(1, len(blk.records)))(*[B.OpRec(f, r, c, n, o) for (f, r, c, o, n) in blk.records])
        data = torch.from_numpy(np.ascontiguousarray(blk.data if blk.data.size else np.zeros(1))).to(device)
        keepalive.extend([sec, rec, data])
        return B.BlockT(len(blk.sectors), 0, ctypes.addressof(sec), len(blk.records), ctypes.addressof(rec),
                        data.data_ptr(), blk.data.size)

    if right_to_left:
        table = list(range(0, grown.p + 1))
        fn = lib.dmrg_sweep_right_to_left
    else:
        table = list(range(grown.p, n_orb - 1))
        fn = lib.dmrg_sweep_left_to_right
    gb = block(grown)
    tb = (B.BlockT * len(table))(*[block(blocks[p]) for p in table])
    steps = (B.SweepStep * len(table))()
    outs = (B.BlockT * len(table))() if keep_blocks else None
    hh = np.ascontiguousarray(h, dtype=np.float64)
    ee = np.ascontiguousarray(eri, dtype=np.float64)
    s = stream if stream is not None else torch.cuda.current_stream(torch.device(device))
    opts = Plan._dav_opts(tol, 1000, 24, 1e-2)
    popts = B.PlanOpts(precision, n_slices, 0, 0, 0, 0, 0, 0, 0, None, None, None, None)
    torch.cuda.synchronize()
    first, second = (tb, ctypes.byref(gb)) if right_to_left else (ctypes.byref(gb), tb)
    B.check(fn(n_orb, n_elec, two_s, hh.ctypes.data, ee.ctypes.data, grown.p, first, second, D,
               ctypes.byref(popts), ctypes.byref(opts), seed, steps, outs, ctypes.c_void_p(s.cuda_stream)), lib)
    res = [(st.bond, st.energy, st.kept, st.kept_weight, st.iters) for st in steps]
    return (res, list(outs)) if keep_blocks else res


def release_blocks(blocks):
    """dmrg_block_release on blocks a sweep returned."""
    lib = B.load()
    for b in blocks:
        lib.dmrg_block_release(ctypes.byref(b))
