"""GPU-side distance of two low-rank density matrices (test helper).

|V1 diag(lam) V1* - V2 diag(lam) V2*|_F / |V2 diag(lam) V2*|_F, formed
without the cancellation of subtracting two nearly equal matrices: with
[V1, V2] = Q R the difference is Q (R D R*) Q*, D = diag(lam, -lam).
"""
import numpy as np


def rel_fro_gpu(V1, V2, lam):
    import torch
    W = torch.cat([V1, V2], dim=1).to(torch.complex128)
    la = torch.as_tensor(np.asarray(lam, dtype=np.float64), device=W.device)
    _, R = torch.linalg.qr(W, mode="r")
    D = torch.cat([la, -la]).to(torch.complex128)
    diff = torch.linalg.norm((R * D[None, :]) @ R.conj().T)
    _, R2 = torch.linalg.qr(V2.to(torch.complex128), mode="r")
    ref = torch.linalg.norm((R2 * la.to(torch.complex128)[None, :]) @ R2.conj().T)
    return float(diff / ref)
