"""Two-state diabatic models for the library (Sec. II.F): the adiabatic surfaces and
coupling that a diabatic potential matrix W(q) implies, the rotation of states between
the two representations, and the items that hand either representation to the GPU.

    V_1,2 = (W11 + W22)/2 +- ((W22 - W11)^2/4 + W12^2)^(1/2)          (Eqs. 24, 26)
    O(q) = rotation by theta, tan(2 theta) = 2 W12 / (W11 - W22)        (Eq. 26)
    F12 = -theta' = ((W22 - W11) W12' - W12 (W22 - W11)') /
          ((W22 - W11)^2 + 4 W12^2)                                      (Eqs. 27, 28)
    psi_adiabatic = O^T psi_diabatic                                     (Eq. 25)

With GQD_SPLIT_OPERATOR the library reads a handle's surfaces as W: V = (W11, W22),
F = W12 (`diabatic_as_surfaces`)."""
from __future__ import annotations

from typing import Tuple

import numpy as np

from .inputs import DiabaticItem, Item1D


def adiabatic_surfaces(W: np.ndarray, dW: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(V of shape (2, n), F12 of shape (n,), theta of shape (n,)) for W = (W11, W22,
    W12) and dW their derivatives; theta lies in (0, pi/2) where W12 > 0."""
    w11, w22, w12 = (np.asarray(x, dtype=np.float64) for x in W)
    d11, d22, d12 = (np.asarray(x, dtype=np.float64) for x in dW)
    gap = w22 - w11
    half = np.hypot(0.5 * gap, w12)
    mean = 0.5 * (w11 + w22)
    V = np.stack([mean + half, mean - half])
    theta = 0.5 * np.arctan2(2.0 * w12, -gap)
    F12 = (gap * d12 - w12 * (d22 - d11)) / (gap * gap + 4.0 * w12 * w12)
    return V, F12, theta


def rotate(psi: np.ndarray, theta: np.ndarray, inverse: bool = False) -> np.ndarray:
    """O^T psi (diabatic -> adiabatic, Eq. 25), or O psi with inverse=True."""
    c, s = np.cos(theta), np.sin(theta)
    if inverse:
        s = -s
    return np.stack([c * psi[0] + s * psi[1], c * psi[1] - s * psi[0]])


def adiabatic_item(d: DiabaticItem) -> Tuple[Item1D, np.ndarray]:
    """The adiabatic item equivalent to d (its state rotated by Eq. 25) and theta."""
    V, F12, theta = adiabatic_surfaces(d.W, d.dW)
    return Item1D(d.n, d.qmin, d.qmax, d.mass, V, F12[None, :], rotate(d.psi0, theta)), theta


def diabatic_as_surfaces(d: DiabaticItem) -> Item1D:
    """d handed to the library for GQD_SPLIT_OPERATOR: V = (W11, W22), F = W12."""
    return Item1D(d.n, d.qmin, d.qmax, d.mass, np.array(d.W[:2]), np.array(d.W[2:3]), d.psi0)
