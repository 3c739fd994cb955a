"""Explicit dense matrices of the paper's operators, for brute-force checks on tiny sizes.

Built straight from the block definitions, independently of the oracle's loops:
BLTT(F_0..F_{Nt-1}) has block (n, m) = F_{n-m} for n >= m and zero above the
diagonal (Sec. II-B3); vectors are stacked time-major, x = [x_0; x_1; ...];
D_t is the backward difference (I - Z)/dt applied to every seafloor point,
Z the one-step delay.
"""
import numpy as np


def bltt_matrix(blocks: np.ndarray) -> np.ndarray:
    """blocks[k] in R^{nout x nin}, k < Nt  ->  dense (Nt*nout) x (Nt*nin) BLTT matrix."""
    nt, nout, nin = blocks.shape
    M = np.zeros((nt * nout, nt * nin))
    for n in range(nt):
        for m in range(n + 1):
            M[n * nout:(n + 1) * nout, m * nin:(m + 1) * nin] = blocks[n - m]
    return M


def dt_matrix(nt: int, npts: int, dt: float, diff: int) -> np.ndarray:
    """Temporal difference on time-major stacked vectors of npts points."""
    if not diff:
        return np.eye(nt * npts)
    Z = np.eye(nt, k=-1)
    return np.kron((np.eye(nt) - Z) / dt, np.eye(npts))


def chain_matrix(G: np.ndarray, F: np.ndarray, dt: float, diff: int) -> np.ndarray:
    """A = BLTT(F_q) D_t BLTT(F_G) for G[g][j][k], F[g][o][k] (storage layouts of the library)."""
    ngrid, nsub, nt = G.shape
    FG = np.transpose(G, (2, 0, 1))          # [k][g][j] = [F_{G,k}]_{g,j}
    FQ = np.transpose(F, (2, 1, 0))          # [k][o][g] = [F_{q,k}]_{o,g}
    return bltt_matrix(FQ) @ dt_matrix(nt, ngrid, dt, diff) @ bltt_matrix(FG)


def to_time_major(x: np.ndarray) -> np.ndarray:
    """[ch][n] -> stacked [n*ch + c]."""
    return np.ascontiguousarray(x.T).reshape(-1)


def from_time_major(v: np.ndarray, nch: int) -> np.ndarray:
    return v.reshape(-1, nch).T.copy()
