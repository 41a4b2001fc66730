"""Closed-form spectra of the constant-coefficient workloads (test pins)."""
import numpy as np


def lap2d_eigs(m):
    """(4/h^2)(sin^2(i pi h/2) + sin^2(j pi h/2)), h = 1/(m+1)."""
    h = 1.0 / (m + 1)
    s = np.sin(np.arange(1, m + 1) * np.pi * h / 2) ** 2
    return np.sort((4.0 / h ** 2 * (s[:, None] + s[None, :])).ravel())


def lap3d_eigs(n, count=None):
    """(4/h^2) sum_d sin^2(i_d pi h/2), h = 1/(n+1)."""
    h = 1.0 / (n + 1)
    s = np.sin(np.arange(1, n + 1) * np.pi * h / 2) ** 2
    m = n if count is None else min(n, count)
    s = s[:m]
    ev = np.sort((4.0 / h ** 2 * (s[:, None, None] + s[None, :, None] + s[None, None, :])).ravel())
    return ev if count is None else ev[:count]


def q1_eigs(n, count=None):
    """(6/h^2) sum_d (1 - cos(i_d pi h)) / (2 + cos(i_d pi h)), h = 1/(n+1)."""
    h = 1.0 / (n + 1)
    c = np.cos(np.arange(1, n + 1) * np.pi * h)
    t = 6.0 / h ** 2 * (1 - c) / (2 + c)
    m = n if count is None else min(n, count)
    t = t[:m]
    ev = np.sort((t[:, None, None] + t[None, :, None] + t[None, None, :]).ravel())
    return ev if count is None else ev[:count]
