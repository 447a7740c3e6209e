"""Helpers for the GPU parity tests: oracle-side references and tensor
conversion.  The oracle (tests' CPU reference) and the HIP library share
nothing; inputs come from `workloads`."""

import numpy as np

from oracle import fem, operators as ops

OP_NAMES = {"B0": ("B", 0.0), "BSHIFT": ("B", None), "L": ("L", None), "N": ("N", None),
            "H": ("H", None), "M": None}


def oracle_matrix(dim, n, op, k, delta_hat):
    K, M, MG = fem.assemble(dim, n)
    if op == "M":
        return M.astype(np.complex128)
    if op == "B0":
        return ops.b_delta(K, M, MG, k, 0.0).tocsr()
    if op == "BSHIFT":
        return ops.b_delta(K, M, MG, k, delta_hat).tocsr()
    if op == "L":
        return ops.hss_lhs(K, M, MG, k, delta_hat).tocsr()
    if op == "N":
        return ops.hss_rhs(K, M, MG, k, delta_hat).tocsr()
    if op == "H":
        return ops.h_gram(M, MG, k, delta_hat).tocsr().astype(np.complex128)
    raise KeyError(op)


def to_dev(a, dtype="complex128"):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to(device="cuda", dtype=getattr(torch, dtype)).contiguous()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.complex128)


def rel_err(a, b):
    """max-norm error relative to the max-norm of the reference b."""
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
