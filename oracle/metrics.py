"""Distance between two low-rank density matrices without cancellation.

||rho_a - rho_b||_F from traces (sum lam^2 + sum mu^2 - 2 sum lam_a mu_b |<a|b>|^2)
cannot resolve differences below ~1e-8.  Instead: QR of [V_a, V_b] = Q R, so
rho_a - rho_b = Q R diag(lam_a, -lam_b) R* Q*, and the Frobenius norm is that
of the small middle matrix.  ||rho_b||_F = ||lam_b||_2 for orthonormal V_b.
"""
import numpy as np
import scipy.linalg as sla


def rho_diff_fro(Va, lam_a, Vb, lam_b):
    Va = np.asarray(Va, dtype=np.complex128)
    Vb = np.asarray(Vb, dtype=np.complex128)
    Q, R = sla.qr(np.concatenate([Va, Vb], axis=1), mode="economic")
    d = np.concatenate([np.asarray(lam_a, np.float64), -np.asarray(lam_b, np.float64)])
    M = (R * d[None, :]) @ R.conj().T
    return float(np.linalg.norm(M))


def rel_fro_error(Va, lam_a, Vb, lam_b):
    """||rho_a - rho_b||_F / ||rho_b||_F with rho = V diag(lam) V*."""
    return rho_diff_fro(Va, lam_a, Vb, lam_b) / float(np.linalg.norm(lam_b))


def dense_rho(V, lam):
    V = np.asarray(V, dtype=np.complex128)
    return (V * np.asarray(lam)[None, :]) @ V.conj().T
