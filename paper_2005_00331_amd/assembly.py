"""Sparse (CSR) assembly of the Jacobian from the library's element matrices.

Not part of the solver path: the products, smoothers and solves are matrix-free.
This assembles the matrix-based operator that Section 6 of the paper compares
the matrix-free product against (memory per dof, product time), on the device:
global dof indices from the documented cell/local-node numbering of
``mfpff_element_matrices``, duplicates summed, 32-bit CSR indices.
"""
import torch


def local_dofs(dim, N, k, device="cuda"):
    """(n_cells, nl) global dofs of every cell's local rows (component, local node)."""
    M = k * N + 1
    nn = M ** dim
    NP = k + 1
    c = torch.arange(N, device=device)
    i = torch.arange(NP, device=device)
    if dim == 2:
        cy, cx = torch.meshgrid(c, c, indexing="ij")
        cells = (k * cx.reshape(-1, 1), k * cy.reshape(-1, 1))
        i1, i0 = torch.meshgrid(i, i, indexing="ij")
        loc = (i0.reshape(1, -1), i1.reshape(1, -1))
        node = (cells[0] + loc[0]) + M * (cells[1] + loc[1])
    else:
        cz, cy, cx = torch.meshgrid(c, c, c, indexing="ij")
        cells = (k * cx.reshape(-1, 1), k * cy.reshape(-1, 1), k * cz.reshape(-1, 1))
        i2, i1, i0 = torch.meshgrid(i, i, i, indexing="ij")
        loc = (i0.reshape(1, -1), i1.reshape(1, -1), i2.reshape(1, -1))
        node = (cells[0] + loc[0]) + M * (cells[1] + loc[1]) + M * M * (cells[2] + loc[2])
    comps = torch.arange(dim + 1, device=device).reshape(1, -1, 1) * nn
    return (comps + node[:, None, :]).reshape(node.shape[0], -1), (dim + 1) * nn


def assemble_csr(em, dim, N, k):
    """CSR (32-bit indices, FP64 values) of sum over cells of the element matrices em
    (n_cells, nl, nl) from ``Context.element_matrices``."""
    ld, n = local_dofs(dim, N, k, em.device)
    nl = ld.shape[1]
    rows = ld[:, :, None].expand(-1, nl, nl).reshape(-1)
    cols = ld[:, None, :].expand(-1, nl, nl).reshape(-1)
    coo = torch.sparse_coo_tensor(torch.stack([rows, cols]), em.reshape(-1), (n, n)).coalesce()
    del rows, cols
    csr = coo.to_sparse_csr()
    del coo
    return torch.sparse_csr_tensor(csr.crow_indices().to(torch.int32), csr.col_indices().to(torch.int32),
                                   csr.values(), (n, n))


class RocsparseSpmv:
    """y = A x with the vendor sparse library (rocSPARSE generic SpMV, FP64, 32-bit CSR
    indices) on torch's current stream; x and y are owned here (``self.x``, ``self.y``)."""

    _ALGS = {"default": 0, "adaptive": 2, "rowsplit": 3, "lrb": 7, "nnzsplit": 8}

    def __init__(self, A, alg="adaptive"):
        import ctypes as C
        import os
        path = "librocsparse.so"
        for d in (os.environ.get("ROCM_PATH", "/opt/rocm") + "/lib", "/opt/rocm/lib"):
            if os.path.exists(os.path.join(d, "librocsparse.so")):
                path = os.path.join(d, "librocsparse.so")
                break
        self.lib = lib = C.CDLL(path)
        self.C = C
        m, n = A.shape
        self.crow, self.col, self.val = A.crow_indices(), A.col_indices(), A.values()
        assert self.crow.dtype == torch.int32 and self.col.dtype == torch.int32 and self.val.dtype == torch.float64
        self.x = torch.zeros(n, dtype=torch.float64, device=self.val.device)
        self.y = torch.zeros(m, dtype=torch.float64, device=self.val.device)
        self.h, self.mat, self.xd, self.yd = C.c_void_p(), C.c_void_p(), C.c_void_p(), C.c_void_p()
        self._ok(lib.rocsparse_create_handle(C.byref(self.h)))
        self._ok(lib.rocsparse_set_stream(self.h, C.c_void_p(torch.cuda.current_stream().cuda_stream)))
        i32, base0, f64 = 2, 0, 152
        self._ok(lib.rocsparse_create_csr_descr(C.byref(self.mat), C.c_int64(m), C.c_int64(n),
                                                C.c_int64(self.val.numel()), C.c_void_p(self.crow.data_ptr()),
                                                C.c_void_p(self.col.data_ptr()), C.c_void_p(self.val.data_ptr()),
                                                C.c_int(i32), C.c_int(i32), C.c_int(base0), C.c_int(f64)))
        self._ok(lib.rocsparse_create_dnvec_descr(C.byref(self.xd), C.c_int64(n), C.c_void_p(self.x.data_ptr()),
                                                  C.c_int(f64)))
        self._ok(lib.rocsparse_create_dnvec_descr(C.byref(self.yd), C.c_int64(m), C.c_void_p(self.y.data_ptr()),
                                                  C.c_int(f64)))
        self.alpha, self.beta = C.c_double(1.0), C.c_double(0.0)
        self.alg = self._ALGS[alg]
        bs = C.c_size_t(0)
        self._spmv(1, C.byref(bs), None)
        self.buf = torch.empty(max(int(bs.value), 1), dtype=torch.uint8, device=self.val.device)
        self.bs = bs
        self._spmv(2, C.byref(self.bs), C.c_void_p(self.buf.data_ptr()))

    def _ok(self, st):
        if st != 0:
            raise RuntimeError(f"rocsparse status {st}")

    def _spmv(self, stage, bs, buf):
        C = self.C
        self._ok(self.lib.rocsparse_spmv(self.h, C.c_int(111), C.byref(self.alpha), self.mat, self.xd,
                                         C.byref(self.beta), self.yd, C.c_int(152), C.c_int(self.alg),
                                         C.c_int(stage), bs, buf))

    def mv(self):
        self._spmv(3, self.C.byref(self.bs), self.C.c_void_p(self.buf.data_ptr()))
        return self.y

    def close(self):
        for f, p in (("rocsparse_destroy_dnvec_descr", self.xd), ("rocsparse_destroy_dnvec_descr", self.yd),
                     ("rocsparse_destroy_spmat_descr", self.mat), ("rocsparse_destroy_handle", self.h)):
            if p:
                getattr(self.lib, f)(p)
        self.xd = self.yd = self.mat = self.h = None
