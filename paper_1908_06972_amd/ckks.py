"""Python front end of libpft: Params / Context / Ciphertext.

Marshalling only: device buffers are torch tensors on the GPU (int64 storage
of uint64 residues), every computation is a libpft call on torch's current
HIP stream.
"""

import ctypes

import numpy as np
import torch

from . import native as N


class Params:
    """SETUP (Sec. 3.4): ring degree, prime chain, special primes, dnum, scale."""

    def __init__(self, log_n, n_q, q0_bits, q_bits, n_p, p_bits, dnum, scale, rescale_mode=0):
        lib = N.load()
        spec = N.ParamSpec(log_n, n_q, q0_bits, q_bits, n_p, p_bits, dnum, rescale_mode, float(scale))
        h = ctypes.c_void_p()
        N.check(lib.pft_params_create(ctypes.byref(spec), ctypes.byref(h)))
        self._adopt(h, log_n, n_q, n_p, dnum, scale)

    def _adopt(self, h, log_n, n_q, n_p, dnum, scale):
        lib = N.load()
        self.handle = h
        self._destroy = lib.pft_params_destroy  # bound now: usable during interpreter shutdown
        self.log_n = log_n
        self.n = 1 << log_n
        self.L = n_q
        self.K = n_p
        self.dnum = dnum
        self.scale = float(scale)
        q = np.zeros(n_q, dtype=np.uint64)
        p = np.zeros(n_p, dtype=np.uint64)
        N.check(lib.pft_params_moduli(h, N.u64p(q), N.u64p(p)))
        self.q = [int(x) for x in q]
        self.p = [int(x) for x in p]
        dims = np.zeros(5, dtype=np.uint32)
        N.check(lib.pft_params_dims(h, dims.ctypes.data_as(N._u32p)))
        self.alpha = int(dims[4])
        mode = ctypes.c_uint32()
        N.check(lib.pft_params_rescale_mode(h, ctypes.byref(mode)))
        self.rescale_mode = mode.value

    @classmethod
    def from_primes(cls, log_n, q, p, dnum, scale, rescale_mode=0):
        """SETUP with the caller's prime chain (pft_params_create_primes)."""
        qa = np.ascontiguousarray(q, dtype=np.uint64)
        pa = np.ascontiguousarray(p, dtype=np.uint64)
        spec = N.ParamPrimes(log_n, len(qa), N.u64p(qa), N.u64p(pa), len(pa), dnum, rescale_mode, 0, float(scale))
        h = ctypes.c_void_p()
        N.check(N.load().pft_params_create_primes(ctypes.byref(spec), ctypes.byref(h)))
        obj = cls.__new__(cls)
        obj._adopt(h, log_n, len(qa), len(pa), dnum, scale)
        return obj

    @classmethod
    def from_config(cls, cfg):
        return cls(cfg.log_n, cfg.n_q, cfg.q0_bits, cfg.q_bits, cfg.n_p, cfg.p_bits, cfg.dnum, cfg.scale)

    def key_moduli(self):
        return self.q + self.p

    def __del__(self):
        if getattr(self, "handle", None) is not None:
            self._destroy(self.handle)
            self.handle = None

    # client-side ENCODE / DECODE on the host
    def encode(self, z, scale=None) -> np.ndarray:
        z = np.asarray(z, dtype=np.complex128)
        re = np.ascontiguousarray(z.real)
        im = np.ascontiguousarray(z.imag)
        out = np.empty(self.n, dtype=np.int64)
        N.check(N.load().pft_encode(self.handle, N.dblp(re), N.dblp(im), len(z),
                                    float(self.scale if scale is None else scale), N.i64p(out)))
        return out

    def diagonals_encode(self, M, n_o, n_i, n_in, scale) -> np.ndarray:
        """Integer plaintexts [n_in][G][b][N] of the pre-rotated diagonals of
        M (n_o x n_in*n_i) at `scale` (client side, host only)."""
        Mc = np.ascontiguousarray(M, dtype=np.float64)
        assert Mc.shape == (n_o, n_in * n_i)
        from .training import bsgs_plan
        b, G = bsgs_plan(n_o, n_in)
        out = np.empty((n_in, G, b, self.n), dtype=np.int64)
        N.check(N.load().pft_diagonals_encode(self.handle, N.dblp(Mc), n_o, n_i, n_in, float(scale), N.i64p(out)))
        return out

    def decode(self, residues, scale, n_slots=None) -> np.ndarray:
        res = np.ascontiguousarray(residues, dtype=np.uint64)
        n_slots = self.n // 2 if n_slots is None else n_slots
        re = np.empty(n_slots)
        im = np.empty(n_slots)
        N.check(N.load().pft_decode(self.handle, N.u64p(res), res.shape[0], float(scale), n_slots,
                                    N.dblp(re), N.dblp(im)))
        return re + 1j * im


class Ciphertext:
    """[2][level][N] residues in the NTT domain, in a torch tensor on the GPU."""

    def __init__(self, data: torch.Tensor, level: int, scale: float):
        self.data = data
        self.level = level
        self.scale = scale

    def desc(self) -> N.CtDesc:
        return N.CtDesc(self.data.data_ptr(), self.level, 0, self.scale)

    def sync_from(self, d: N.CtDesc):
        self.level = d.level
        self.scale = d.scale
        return self


class Plaintext(Ciphertext):
    """[level][N] NTT-domain plaintext on the GPU."""


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


class TorchAllocator:
    """Device memory for the library's own buffers from torch's caching
    allocator (pft_allocator callbacks), on the context's stream."""

    def __init__(self, stream):
        self.stream = stream
        self.live = {}

        def alloc(_user, nbytes, device):
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), device, self.stream)
            except RuntimeError:
                return None
            self.live[ptr] = int(nbytes)
            return ptr

        def free(_user, ptr):
            if ptr in self.live:
                del self.live[ptr]
                torch.cuda.caching_allocator_delete(ptr)

        self.alloc_fn = N.ALLOC_FN(alloc)
        self.free_fn = N.FREE_FN(free)


class Context:
    def __init__(self, params: Params, device: int = 0, stream=None, budget_bytes=0, torch_memory=False):
        """stream: a torch.cuda.Stream to run on (default: torch's current
        stream).  Graph capture needs a stream other than the null stream.
        budget_bytes: cap on the library's own device memory (0: none);
        torch_memory: take that memory from torch's caching allocator."""
        self.params = params
        self.device = torch.device("cuda", device)
        self.lib = N.load()
        h = ctypes.c_void_p()
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        stream = self.stream.cuda_stream
        self._alloc = None
        if budget_bytes or torch_memory:
            spec = N.Allocator()
            if torch_memory:
                self._alloc = TorchAllocator(self.stream)
                spec.alloc, spec.free = self._alloc.alloc_fn, self._alloc.free_fn
            spec.budget_bytes = int(budget_bytes)
            N.check(self.lib.pft_ctx_create_alloc(params.handle, device, ctypes.c_void_p(stream), ctypes.byref(spec),
                                                  ctypes.byref(h)))
        else:
            N.check(self.lib.pft_ctx_create(params.handle, device, ctypes.c_void_p(stream), ctypes.byref(h)))
        self.handle = h

    def set_budget(self, budget_bytes):
        N.check(self.lib.pft_ctx_set_budget(self.handle, int(budget_bytes)))

    def memory(self):
        """{"tables_keys", "scratch", "budget"} device bytes of the library's own buffers."""
        out = np.zeros(3, dtype=np.uint64)
        N.check(self.lib.pft_ctx_memory(self.handle, N.u64p(out)))
        return dict(zip(("tables_keys", "scratch", "budget"), (int(x) for x in out)))

    def close(self):
        if getattr(self, "handle", None) is not None:
            self.lib.pft_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()

    def synchronize(self):
        N.check(self.lib.pft_ctx_synchronize(self.handle))

    def reserve(self, ws_bytes, aux_bytes=0):
        N.check(self.lib.pft_ctx_reserve(self.handle, int(ws_bytes), int(aux_bytes)))

    def capture(self, fn):
        """Record the libpft calls made by fn() into a HIP graph (fn must pass
        preallocated outputs: nothing may allocate while capturing)."""
        N.check(self.lib.pft_graph_begin(self.handle))
        try:
            fn()
        except Exception:
            h = ctypes.c_void_p()
            self.lib.pft_graph_end(self.handle, ctypes.byref(h))
            if h.value:
                self.lib.pft_graph_destroy(h)
            raise
        h = ctypes.c_void_p()
        N.check(self.lib.pft_graph_end(self.handle, ctypes.byref(h)))
        return Graph(self, h)

    def device_bytes(self) -> int:
        b = ctypes.c_uint64()
        N.check(self.lib.pft_ctx_device_bytes(self.handle, ctypes.byref(b)))
        return b.value

    # ---- buffers
    def empty_ct(self, level: int, scale: float = 0.0) -> Ciphertext:
        # allocated on the context stream, so the caching allocator orders reuse with its work
        with torch.cuda.stream(self.stream):
            t = torch.empty((2, level, self.params.n), dtype=torch.int64, device=self.device)
        return Ciphertext(t, level, scale)

    def empty_pt(self, level: int) -> Plaintext:
        with torch.cuda.stream(self.stream):
            t = torch.empty((level, self.params.n), dtype=torch.int64, device=self.device)
        return Plaintext(t, level, 0.0)

    # ---- KEYGEN (randomness as arguments)
    def set_secret(self, s):
        N.check(self.lib.pft_set_secret(self.handle, N.i64p(_i64(s))))

    def gen_public_key(self, a, e):
        N.check(self.lib.pft_gen_public_key(self.handle, N.u64p(_u64(a)), N.i64p(_i64(e))))

    def gen_relin_key(self, a, e):
        N.check(self.lib.pft_gen_relin_key(self.handle, N.u64p(_u64(a)), N.i64p(_i64(e))))

    def set_key_cache(self, max_resident: int):
        """Keep at most max_resident rotation keys on the device (0: all);
        the others live in pinned host memory and are copied in on use."""
        N.check(self.lib.pft_set_key_cache(self.handle, int(max_resident)))

    def key_cache_plan(self, steps):
        """Expected cyclic order of rotation steps (eviction and copy-ahead)."""
        arr = np.ascontiguousarray(np.asarray(list(steps), dtype=np.int32))
        N.check(self.lib.pft_key_cache_plan(self.handle, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            int(arr.size)))

    def key_cache_stats(self):
        out = np.zeros(6, dtype=np.uint64)
        N.check(self.lib.pft_key_cache_stats(self.handle, N.u64p(out)))
        return dict(zip(("max_resident", "slots", "hits", "misses", "bytes_in", "prefetches"),
                        (int(x) for x in out)))

    def gen_rotation_key(self, step, a, e):
        N.check(self.lib.pft_gen_rotation_key(self.handle, int(step), N.u64p(_u64(a)), N.i64p(_i64(e))))

    def keygen(self, seed, rot_steps=()):
        """Secret, public, relinearisation and rotation keys (one per step),
        every draw taken on the device from the Philox streams of `seed`."""
        steps = (ctypes.c_int32 * max(1, len(rot_steps)))(*[int(s) for s in rot_steps])
        N.check(self.lib.pft_keygen(self.handle, ctypes.c_uint64(int(seed)), steps, len(rot_steps)))

    # ---- ENC / DEC
    def encrypt(self, m, level, scale, v, e0, e1) -> Ciphertext:
        ct = self.empty_ct(level)
        d = ct.desc()
        N.check(self.lib.pft_encrypt(self.handle, N.i64p(_i64(m)), level, float(scale), N.i64p(_i64(v)),
                                     N.i64p(_i64(e0)), N.i64p(_i64(e1)), ctypes.byref(d)))
        return ct.sync_from(d)

    def encrypt_seeded(self, m, level, scale, seed) -> Ciphertext:
        """ENC with v, e0, e1 drawn on the device from the streams of `seed`."""
        ct = self.empty_ct(level)
        d = ct.desc()
        N.check(self.lib.pft_encrypt_seeded(self.handle, N.i64p(_i64(m)), level, float(scale),
                                            ctypes.c_uint64(int(seed)), ctypes.byref(d)))
        return ct.sync_from(d)

    def decrypt(self, ct: Ciphertext) -> np.ndarray:
        out = np.empty((ct.level, self.params.n), dtype=np.uint64)
        d = ct.desc()
        N.check(self.lib.pft_decrypt(self.handle, ctypes.byref(d), N.u64p(out)))
        return out

    def export(self, ct: Ciphertext) -> np.ndarray:
        out = np.empty((2, ct.level, self.params.n), dtype=np.uint64)
        d = ct.desc()
        N.check(self.lib.pft_ct_export(self.handle, ctypes.byref(d), N.u64p(out)))
        return out

    def import_(self, host, level, scale) -> Ciphertext:
        ct = self.empty_ct(level)
        d = ct.desc()
        N.check(self.lib.pft_ct_import(self.handle, N.u64p(_u64(host)), level, float(scale), ctypes.byref(d)))
        return ct.sync_from(d)

    def plaintext(self, m, level, scale) -> Plaintext:
        pt = self.empty_pt(level)
        d = pt.desc()
        N.check(self.lib.pft_pt_from_coeffs(self.handle, N.i64p(_i64(m)), level, float(scale), ctypes.byref(d)))
        return pt.sync_from(d)

    # ---- homomorphic operations
    def _binary(self, fn, a, b, out):
        da, db, do = a.desc(), b.desc(), out.desc()
        N.check(fn(self.handle, ctypes.byref(da), ctypes.byref(db), ctypes.byref(do)))
        return out.sync_from(do)

    def add(self, a, b, out=None):
        return self._binary(self.lib.pft_add, a, b, out or self.empty_ct(a.level))

    def add_plain(self, a, p, out=None):
        return self._binary(self.lib.pft_add_plain, a, p, out or self.empty_ct(a.level))

    def mul_plain(self, a, p, out=None):
        return self._binary(self.lib.pft_mul_plain, a, p, out or self.empty_ct(a.level))

    def mul_relin(self, a, b, out=None):
        return self._binary(self.lib.pft_mul_relin, a, b, out or self.empty_ct(a.level))

    def _arr(self, cts):
        arr = (N.CtDesc * len(cts))()
        for i, c in enumerate(cts):
            arr[i] = c.desc()
        return arr

    def mul_relin_batch(self, a, b, out=None):
        out = out or [self.empty_ct(x.level) for x in a]
        A, B, O = self._arr(a), self._arr(b), self._arr(out)
        N.check(self.lib.pft_mul_relin_batch(self.handle, len(a), A, B, O))
        return [o.sync_from(O[i]) for i, o in enumerate(out)]

    def mul_relin_batch_noalloc(self, a, b, out):
        """mul_relin_batch with the workspace in the library's fixed device
        scratch: no device allocation in the call (outputs must be given)."""
        A, B, O = self._arr(a), self._arr(b), self._arr(out)
        N.check(self.lib.pft_mul_relin_batch_noalloc(self.handle, len(a), A, B, O))
        return [o.sync_from(O[i]) for i, o in enumerate(out)]

    def rescale(self, a, mode=0, out=None):
        out = out or self.empty_ct(a.level - 1)
        da, do = a.desc(), out.desc()
        N.check(self.lib.pft_rescale(self.handle, ctypes.byref(da), mode, ctypes.byref(do)))
        return out.sync_from(do)

    def rescale_batch(self, a, mode=0, out=None):
        out = out or [self.empty_ct(x.level - 1) for x in a]
        A, O = self._arr(a), self._arr(out)
        N.check(self.lib.pft_rescale_batch(self.handle, len(a), A, mode, O))
        return [o.sync_from(O[i]) for i, o in enumerate(out)]

    def mod_drop(self, a, level, out=None):
        out = out or self.empty_ct(level)
        da, do = a.desc(), out.desc()
        N.check(self.lib.pft_mod_drop(self.handle, ctypes.byref(da), level, ctypes.byref(do)))
        return out.sync_from(do)

    def rotate(self, a, step, out=None):
        out = out or self.empty_ct(a.level)
        da, do = a.desc(), out.desc()
        N.check(self.lib.pft_rotate(self.handle, ctypes.byref(da), int(step), ctypes.byref(do)))
        return out.sync_from(do)

    def exec_batch(self, cts, ops):
        """Run an op list (see pft_exec_batch) over the ciphertexts `cts`.
        ops: tuples (kind, a, b, out, step, mode) with kind one of
        'ntt', 'intt', 'add', 'mul_relin', 'rescale', 'rotate' and a/b/out
        indices into cts (unused fields may be 0).  Output ciphertexts must be
        allocated for their level; levels and scales are updated in place."""
        kinds = {"ntt": N.PFT_OP_NTT, "intt": N.PFT_OP_INTT, "add": N.PFT_OP_ADD, "mul_relin": N.PFT_OP_MUL_RELIN,
                 "rescale": N.PFT_OP_RESCALE, "rotate": N.PFT_OP_ROTATE}
        C = self._arr(cts)
        O = (N.OpDesc * len(ops))()
        for i, (kind, a, b, out, step, mode) in enumerate(ops):
            O[i] = N.OpDesc(kinds[kind], a, b, out, int(step), mode)
        N.check(self.lib.pft_exec_batch(self.handle, C, len(cts), O, len(ops)))
        for i, c in enumerate(cts):
            c.sync_from(C[i])
        return cts

    def rotate_pow2(self, a, step, out=None):
        """Rotation by step from the power-of-two keys of its binary expansion."""
        out = out or self.empty_ct(a.level)
        da, do = a.desc(), out.desc()
        N.check(self.lib.pft_rotate_pow2(self.handle, ctypes.byref(da), int(step), ctypes.byref(do)))
        return out.sync_from(do)

    def rotate_pow2_batch(self, a, step, out=None):
        out = out or [self.empty_ct(x.level) for x in a]
        A, O = self._arr(a), self._arr(out)
        N.check(self.lib.pft_rotate_pow2_batch(self.handle, len(a), A, int(step), O))
        return [o.sync_from(O[i]) for i, o in enumerate(out)]

    def rotate_batch(self, a, step, out=None):
        out = out or [self.empty_ct(x.level) for x in a]
        A, O = self._arr(a), self._arr(out)
        N.check(self.lib.pft_rotate_batch(self.handle, len(a), A, int(step), O))
        return [o.sync_from(O[i]) for i, o in enumerate(out)]

    def total_sum(self, a, n_slots, out=None):
        out = out or self.empty_ct(a.level)
        da, do = a.desc(), out.desc()
        N.check(self.lib.pft_total_sum(self.handle, ctypes.byref(da), n_slots, ctypes.byref(do)))
        return out.sync_from(do)

    def total_sum_batch(self, a, n_slots, out=None):
        out = out or [self.empty_ct(x.level) for x in a]
        A, O = self._arr(a), self._arr(out)
        N.check(self.lib.pft_total_sum_batch(self.handle, len(a), A, n_slots, O))
        return [o.sync_from(O[i]) for i, o in enumerate(out)]

    def mul_const_batch(self, a, values, out=None):
        out = out or [self.empty_ct(x.level) for x in a]
        A, O = self._arr(a), self._arr(out)
        vals = np.ascontiguousarray(values, dtype=np.float64)
        N.check(self.lib.pft_mul_const_batch(self.handle, len(a), A, N.dblp(vals), O))
        return [o.sync_from(O[i]) for i, o in enumerate(out)]

    def add_const_batch(self, a, values, out=None):
        out = out or [self.empty_ct(x.level) for x in a]
        A, O = self._arr(a), self._arr(out)
        vals = np.ascontiguousarray(values, dtype=np.float64)
        N.check(self.lib.pft_add_const_batch(self.handle, len(a), A, N.dblp(vals), O))
        return [o.sync_from(O[i]) for i, o in enumerate(out)]

    def ctmatvec(self, diags, n_o, n_i, n_in, inputs, out=None):
        """Encrypted matrix x encrypted vector.  diags: flat list of
        n_in * G * b ciphertexts in [n_in][G][b] order; inputs: list over
        documents of lists of n_in ciphertexts."""
        flat = [c for doc in inputs for c in doc]
        out = out or [self.empty_ct(doc[0].level) for doc in inputs]
        D, A, O = self._arr(diags), self._arr(flat), self._arr(out)
        N.check(self.lib.pft_ctmatvec(self.handle, n_o, n_i, n_in, D, len(inputs), A, O))
        return [o.sync_from(O[i]) for i, o in enumerate(out)]

    def ptdot(self, slots, level):
        """Plaintexts P[k][j] from slot vectors [n_out][J][t] (library encoder,
        scale q_{level-1})."""
        sl = np.ascontiguousarray(slots, dtype=np.float64)
        n_out, J, t = sl.shape
        assert t == self.params.n // 2
        h = ctypes.c_void_p()
        N.check(self.lib.pft_ptdot_create(self.handle, N.dblp(sl), n_out, J, level, ctypes.byref(h)))
        return PtDot(self, h, n_out, J, level)

    def ptdot_from_coeffs(self, coeffs, level, pt_scale):
        """Plaintexts P[k][j] from integer polynomials [n_out][J][N]."""
        c = np.ascontiguousarray(coeffs, dtype=np.int64)
        n_out, J, n = c.shape
        assert n == self.params.n
        h = ctypes.c_void_p()
        N.check(self.lib.pft_ptdot_create_from_coeffs(self.handle, N.i64p(c), n_out, J, level, float(pt_scale),
                                                      ctypes.byref(h)))
        return PtDot(self, h, n_out, J, level)

    def ptdot_apply(self, mat, inputs, n_sum=1, out=None):
        """inputs: list over documents of lists of J ciphertexts; returns per
        document a list of n_out ciphertexts."""
        flat = [c for doc in inputs for c in doc]
        outs = out or [self.empty_ct(mat.level) for _ in range(len(inputs) * mat.n_out)]
        A, O = self._arr(flat), self._arr(outs)
        N.check(self.lib.pft_ptdot_apply(self.handle, mat.handle, len(inputs), A, int(n_sum), O))
        res = [o.sync_from(O[i]) for i, o in enumerate(outs)]
        return [res[d * mat.n_out:(d + 1) * mat.n_out] for d in range(len(inputs))]

    def ptmat(self, M, n_o, n_i, n_in, level):
        """Plaintext matrix from doubles (library encoder)."""
        h = ctypes.c_void_p()
        Mc = np.ascontiguousarray(M, dtype=np.float64)
        assert Mc.shape == (n_o, n_in * n_i)
        N.check(self.lib.pft_ptmat_create(self.handle, N.dblp(Mc), n_o, n_i, n_in, level, ctypes.byref(h)))
        return PtMat(self, h)

    def ptmat_from_coeffs(self, coeffs, n_o, n_i, n_in, level, pt_scale):
        """Plaintext matrix from integer plaintexts [n_in][G][b][N]."""
        h = ctypes.c_void_p()
        c = np.ascontiguousarray(coeffs, dtype=np.int64)
        N.check(self.lib.pft_ptmat_create_from_coeffs(self.handle, N.i64p(c), n_o, n_i, n_in, level,
                                                      float(pt_scale), ctypes.byref(h)))
        return PtMat(self, h)

    def ptmatvec(self, mat, inputs, out=None):
        """inputs: list over documents of lists of n_in ciphertexts."""
        flat = [c for doc in inputs for c in doc]
        out = out or [self.empty_ct(doc[0].level) for doc in inputs]
        A, O = self._arr(flat), self._arr(out)
        N.check(self.lib.pft_ptmatvec(self.handle, mat.handle, len(inputs), A, O))
        return [o.sync_from(O[i]) for i, o in enumerate(out)]

    def ntt_forward(self, data: torch.Tensor, n_limbs: int):
        n_polys = data.numel() // (n_limbs * self.params.n)
        N.check(self.lib.pft_ntt_forward(self.handle, ctypes.c_void_p(data.data_ptr()), n_polys, n_limbs))

    def ntt_inverse(self, data: torch.Tensor, n_limbs: int):
        n_polys = data.numel() // (n_limbs * self.params.n)
        N.check(self.lib.pft_ntt_inverse(self.handle, ctypes.c_void_p(data.data_ptr()), n_polys, n_limbs))

    # ---- NTT pass schedules (see pft_ntt_candidates): a schedule is
    # (radices in forward order, flags) with flag 1 = the last window's pass
    # skips the LDS staging, flag 2 = 8 residues per thread instead of 16
    @staticmethod
    def _sched_from(words):
        return tuple(int(r) for r in words[:3] if r), int(words[3])

    @staticmethod
    def _sched_to(sched):
        radices, flags = sched
        return (ctypes.c_uint32 * 4)(*(list(radices) + [0] * (3 - len(radices)) + [int(flags)]))

    def ntt_candidates(self):
        n = self.lib.pft_ntt_candidates(self.params.handle, None, 0)
        if n < 0:
            N.check(n)
        buf = (ctypes.c_uint32 * (4 * n))()
        self.lib.pft_ntt_candidates(self.params.handle, buf, n)
        return [self._sched_from(buf[4 * i:4 * i + 4]) for i in range(n)]

    def bconv_mode(self, mfma: bool, fused: bool = True, inner: bool = True, pairs: bool = True):
        """Base conversions on the matrix cores (True, the default) or the
        VALU; with `fused` (the default) the conversions also apply the
        adjacent passes of the transforms, and with `inner` (the default,
        needs `fused`) the key inner product runs in the row pass of ModUp's
        rows, two digits per row pass with `pairs` (pft_bconv_mode 3, the
        default) or one (mode 4)."""
        mode = ((3 if pairs else 4) if inner else 2) if fused else 1
        N.check(self.lib.pft_bconv_mode(self.handle, mode if mfma else 0))

    def ntt_autotune(self, enable: bool):
        N.check(self.lib.pft_ntt_autotune(self.handle, int(bool(enable))))

    def ntt_set_schedule(self, inverse: bool, sched):
        """sched: (radices, flags), or None to unpin."""
        arr = None if sched is None else self._sched_to(sched)
        N.check(self.lib.pft_ntt_set_schedule(self.handle, int(bool(inverse)), arr))

    def ntt_tuning_export(self):
        """Tuned choices: list of (inverse, class, (radices, flags))."""
        n = self.lib.pft_ntt_tuning_export(self.handle, None, 0)
        if n < 0:
            N.check(n)
        buf = (ctypes.c_uint32 * (6 * max(n, 1)))()
        self.lib.pft_ntt_tuning_export(self.handle, buf, n)
        return [(bool(buf[6 * i]), int(buf[6 * i + 1]), self._sched_from(buf[6 * i + 2:6 * i + 6])) for i in range(n)]

    def ntt_tuning_import(self, table):
        buf = (ctypes.c_uint32 * (6 * max(len(table), 1)))()
        for i, (inv, cls, sched) in enumerate(table):
            buf[6 * i] = int(bool(inv))
            buf[6 * i + 1] = int(cls)
            for k, w in enumerate(self._sched_to(sched)):
                buf[6 * i + 2 + k] = w
        N.check(self.lib.pft_ntt_tuning_import(self.handle, buf, len(table)))

    def ntt_get_schedule(self, inverse: bool, n_limbs: int):
        arr = (ctypes.c_uint32 * 4)()
        N.check(self.lib.pft_ntt_get_schedule(self.handle, int(bool(inverse)), n_limbs, arr))
        return self._sched_from(arr)


class Graph:
    def __init__(self, ctx, handle):
        self.ctx = ctx
        self.handle = handle

    def launch(self):
        N.check(self.ctx.lib.pft_graph_launch(self.ctx.handle, self.handle))

    def close(self):
        if getattr(self, "handle", None) is not None:
            self.ctx.lib.pft_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


OP_NAMES = {N.PFT_OP_ROTATE: "rotate", N.PFT_OP_MUL_PLAIN: "mul_plain", N.PFT_OP_ADD: "add"}


def _plan_list(buf, n):
    return [(OP_NAMES[buf[i].kind], buf[i].a, buf[i].b, buf[i].out, buf[i].step) for i in range(n)]


def ptmat_plan(n_o, n_i, n_in):
    """The PtMatVec op list of a shape (pft_ptmat_plan): tuples
    (kind, a, b, out, step) with kind 'rotate', 'mul_plain' or 'add'."""
    lib = N.load()
    cnt = ctypes.c_uint32()
    N.check(lib.pft_ptmat_plan(n_o, n_i, n_in, None, 0, ctypes.byref(cnt)))
    buf = (N.OpDesc * max(cnt.value, 1))()
    N.check(lib.pft_ptmat_plan(n_o, n_i, n_in, buf, cnt.value, ctypes.byref(cnt)))
    return _plan_list(buf, cnt.value)


class PtMat:
    def __init__(self, ctx, handle):
        self.ctx = ctx
        self.handle = handle
        info = np.zeros(6, dtype=np.uint32)
        N.check(ctx.lib.pft_ptmat_info(handle, info.ctypes.data_as(N._u32p)))
        self.n_o, self.n_i, self.n_in, self.level, self.b, self.G = (int(x) for x in info)

    def plan_export(self):
        """(op list as ptmat_plan, integer plaintexts [n_in][G][b][N])."""
        lib = self.ctx.lib
        cnt = ctypes.c_uint32()
        N.check(lib.pft_ptmat_plan_export(self.handle, None, 0, ctypes.byref(cnt), None))
        buf = (N.OpDesc * max(cnt.value, 1))()
        coeffs = np.empty((self.n_in, self.G, self.b, self.ctx.params.n), dtype=np.int64)
        N.check(lib.pft_ptmat_plan_export(self.handle, buf, cnt.value, ctypes.byref(cnt), N.i64p(coeffs)))
        return _plan_list(buf, cnt.value), coeffs

    def __del__(self):
        if getattr(self, "handle", None) is not None:
            self.ctx.lib.pft_ptmat_destroy(self.handle)
            self.handle = None


class PtDot:
    """n_out groups of J plaintexts for pft_ptdot_apply."""

    def __init__(self, ctx, handle, n_out, J, level):
        self.ctx, self.handle = ctx, handle
        self.n_out, self.J, self.level = n_out, J, level

    def __del__(self):
        if getattr(self, "handle", None) is not None:
            self.ctx.lib.pft_ptdot_destroy(self.handle)
            self.handle = None


def to_device_u64(a: np.ndarray, device) -> torch.Tensor:
    """Host uint64 array -> GPU int64 tensor with the same bits."""
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to(device)


def to_host_u64(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)
