"""Shared helpers for the device-vs-oracle parity tests."""
from __future__ import annotations

import numpy as np


def rel_err(x, ref, floor):
    """Max-norm error scaled by max(|ref|_inf, floor) (floors keep near-zero
    fields such as the spurious velocity of a resting drop well posed)."""
    x = np.asarray(x, float)
    ref = np.asarray(ref, float)
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), floor))


def field_floors(inst):
    ph = inst.phys
    meta = inst.meta
    if meta.get("kind") == "droplet":
        u_char = np.sqrt(max(ph.sigma, 1e-12) / (ph.rho_l * meta["radius"]))
        p_char = max(meta["dp_laplace"], 1e-12)
    elif meta.get("kind") == "channel":
        u_char = max(float(np.abs(inst.u0).max()), 1e-12)
        # driven flow: hydrostatic or dynamic pressure, whichever is larger
        p_char = max(ph.rho_l * abs(meta["g"]) * 2 * meta["half_width"], ph.rho_l * u_char ** 2)
    else:
        g = np.linalg.norm(ph.grav)
        u_char = np.sqrt(max(g, 1e-12) * np.ptp(inst.mesh["xyz"][:, 0]))
        p_char = ph.rho_l * max(g, 1e-12) * np.ptp(inst.mesh["xyz"][:, 1])
    return dict(rho=ph.rho_l, C=1.0, u=u_char, p=p_char)


def compare_fields(dev, orc, inst):
    fl = field_floors(inst)
    return {k: rel_err(dev[k], orc[k], fl[k]) for k in ("rho", "u", "p", "C")}
