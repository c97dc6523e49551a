"""Helpers shared by the GPU parity tests (no method arithmetic)."""
import numpy as np
import scipy.sparse as sp


def bsr_to_csr(ctx, blocks):
    """[nnzb,4,4] blocks on the node pattern -> 4N x 4N field-split CSR."""
    rp, col = ctx.pattern()
    N = ctx.N
    B = blocks.detach().cpu().numpy()
    rows = np.repeat(np.arange(N), np.diff(rp))
    gi = np.concatenate([3 * rows[:, None] + np.arange(3)[None, :], (3 * N + rows)[:, None]], axis=1)  # [nnzb,4]
    gj = np.concatenate([3 * col[:, None] + np.arange(3)[None, :], (3 * N + col)[:, None]], axis=1)
    R = np.broadcast_to(gi[:, :, None], B.shape).ravel()
    Cc = np.broadcast_to(gj[:, None, :], B.shape).ravel()
    M = sp.coo_matrix((B.ravel(), (R, Cc)), shape=(4 * N, 4 * N)).tocsr()
    M.sum_duplicates()
    return M


def oracle_full(S):
    """Oracle F-part of the tangent as 4N x 4N CSR (rank-one term excluded)."""
    return sp.bmat([[S.A_F, S.B], [S.C, S.D]]).tocsr()


def block_rel_err(Mg, Mo, n3):
    """max |diff| / max |oracle| per block A, B, C, D."""
    out = {}
    D = (Mg - Mo).tocsr()
    for name, rs, cs in [("A", slice(0, n3), slice(0, n3)), ("B", slice(0, n3), slice(n3, None)),
                         ("C", slice(n3, None), slice(0, n3)), ("D", slice(n3, None), slice(n3, None))]:
        den = abs(Mo[rs, cs]).max()
        num = abs(D[rs, cs]).max() if D[rs, cs].nnz else 0.0
        out[name] = num / den if den > 0 else num
    return out


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
