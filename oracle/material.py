"""Compressible Neo-Hookean hyperelasticity (paper Sec. 6.1).

    W(F) = lambda/2 (ln J)^2 - mu ln J + mu/2 (tr C - 3),  C = F^T F,  J = det F > 0.

The paper prints W only.  Its derivatives, written out here, are
    P = dW/dF = mu F + (lambda ln J - mu) F^{-T}
    A_iJkL = dP_iJ/dF_kL
           = mu d_ik d_JL + lambda Finv_Ji Finv_Lk + (mu - lambda ln J) Finv_Jk Finv_Li
(using d(ln J)/dF = F^{-T} and d(Finv_Ji)/dF_kL = -Finv_Jk Finv_Li).

Tensors are arrays [..., 3, 3]; the 9x9 matrix of A uses the row-major vector
of a 2-tensor (index 3 i + J, paper Sec. 1.5 notation).
"""
import numpy as np


def energy(F, mu, lam):
    """W(F) of paper Sec. 6.1."""
    J = np.linalg.det(F)
    C = np.einsum("...ki,...kj->...ij", F, F)
    lnJ = np.log(J)
    return 0.5 * lam * lnJ ** 2 - mu * lnJ + 0.5 * mu * (np.trace(C, axis1=-2, axis2=-1) - 3.0)


def stress(F, mu, lam):
    """First Piola-Kirchhoff stress P = dW/dF."""
    J = np.linalg.det(F)
    FinvT = np.swapaxes(np.linalg.inv(F), -1, -2)
    lnJ = np.log(J)[..., None, None]
    mu_ = np.asarray(mu)[..., None, None] if np.ndim(mu) else mu
    lam_ = np.asarray(lam)[..., None, None] if np.ndim(lam) else lam
    return mu_ * F + (lam_ * lnJ - mu_) * FinvT


def tangent(F, mu, lam):
    """A = dP/dF as a 9x9 matrix per point, rows 3i+J, columns 3k+L."""
    J = np.linalg.det(F)
    Fi = np.linalg.inv(F)                      # Fi[J, i] = Finv_Ji
    lnJ = np.log(J)
    mu_ = np.asarray(mu, float)
    lam_ = np.asarray(lam, float)
    eye = np.eye(3)
    # term 1: mu d_ik d_JL
    t1 = np.einsum("ik,JL->iJkL", eye, eye)
    # term 2: lambda Finv_Ji Finv_Lk
    t2 = np.einsum("...Ji,...Lk->...iJkL", Fi, Fi)
    # term 3: (mu - lambda ln J) Finv_Jk Finv_Li
    t3 = np.einsum("...Jk,...Li->...iJkL", Fi, Fi)
    m = mu_ - lam_ * lnJ
    A = (mu_[..., None, None, None, None] * t1
         + lam_[..., None, None, None, None] * t2
         + m[..., None, None, None, None] * t3) if np.ndim(m) else (mu_ * t1 + lam_ * t2 + m * t3)
    return A.reshape(A.shape[:-4] + (9, 9))


def isotropic_stiffness(mu, lam):
    """Small-strain isotropic stiffness lambda I(x)I + mu (d_ik d_JL + d_iL d_Jk), as 9x9.

    Textbook linear elasticity; the Neo-Hookean tangent at F = I must equal it."""
    eye = np.eye(3)
    C = (lam * np.einsum("iJ,kL->iJkL", eye, eye)
         + mu * (np.einsum("ik,JL->iJkL", eye, eye) + np.einsum("iL,Jk->iJkL", eye, eye)))
    return C.reshape(9, 9)


def linear_stress(F, mu, lam):
    """Small-strain isotropic law sigma = lambda tr(eps) I + 2 mu eps with
    eps = sym(H), H = F - I the displacement gradient (infinitesimal strain
    theory of the appendix cheat sheet; the stiffness is isotropic_stiffness)."""
    H = F - np.eye(3)
    eps = 0.5 * (H + np.swapaxes(H, -1, -2))
    tr = np.trace(eps, axis1=-2, axis2=-1)[..., None, None]
    return lam * tr * np.eye(3) + 2.0 * mu * eps
