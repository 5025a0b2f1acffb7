"""Shared helpers for the device-vs-oracle parity tests.

Error norm: max |x_dev - x_oracle| / max(|x_oracle|_inf, floor_x), with the
floors of the error-norm reading (the tolerances name no norm): rho -> rho_l,
C -> 1, p -> the configuration's pressure scale (Laplace jump for drops,
hydrostatic or dynamic pressure for the channel, the Laplace jump or the
dynamic pressure for the pipe, rho_l g H for Rayleigh-Taylor), u -> its
characteristic speed (sqrt(sigma / (rho_l R)) for drops, the imposed speed
for translated drops, the peak of the inflow profile for the channel and
the pipe, sqrt(g W) for Rayleigh-Taylor).  The velocity of a
resting drop is a spurious current, the small residual of forcing terms
that nearly cancel, so without a floor its relative error is ill posed.

compare_fields also returns "u_rel" = max |u_dev - u_oracle| / max|u_oracle|,
the velocity error with no floor, which tests report and bound separately
(see velocity_bound).
"""
from __future__ import annotations

import numpy as np

def rel_err(x, ref, floor):
    """Max-norm error scaled by max(|ref|_inf, floor)."""
    x = np.asarray(x, float)
    ref = np.asarray(ref, float)
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), floor))


def characteristic_speed(inst):
    ph = inst.phys
    meta = inst.meta
    kind = meta.get("kind")
    if kind == "translation":
        return float(np.linalg.norm(meta["u0"]))
    if kind == "droplet":
        return float(np.sqrt(max(ph.sigma, 1e-12) / (ph.rho_l * meta["radius"])))
    if kind in ("channel", "pipe"):
        return max(float(np.abs(inst.u0).max()), 1e-12)
    g = np.linalg.norm(ph.grav)
    return float(np.sqrt(max(g, 1e-12) * np.ptp(inst.mesh["xyz"][:, 0])))


def field_floors(inst):
    ph = inst.phys
    meta = inst.meta
    kind = meta.get("kind")
    u_char = characteristic_speed(inst)
    if kind in ("droplet", "translation"):
        p_char = max(meta["dp_laplace"], 1e-12)
    elif kind == "channel":
        # driven flow: hydrostatic or dynamic pressure, whichever is larger
        p_char = max(ph.rho_l * abs(meta["g"]) * 2 * meta["half_width"], ph.rho_l * u_char ** 2)
    elif kind == "pipe":
        # axial flow: the Laplace jump of the cylindrical interface or the dynamic pressure
        p_char = max(meta["dp_laplace"], ph.rho_l * u_char ** 2)
    else:
        g = np.linalg.norm(ph.grav)
        p_char = ph.rho_l * max(g, 1e-12) * np.ptp(inst.mesh["xyz"][:, 1])
    return dict(rho=ph.rho_l, C=1.0, u=u_char, p=p_char)


def compare_fields(dev, orc, inst):
    fl = field_floors(inst)
    out = {k: rel_err(dev[k], orc[k], fl[k]) for k in ("rho", "u", "p", "C")}
    out["u_rel"] = rel_err(dev["u"], orc["u"], 1e-300)
    return out


# FP16 deviation storage (precision FEL_PREC_FP32_FP16): every population is
# stored as psi_a = w_a (ref + s d_a) with d_a in FP16 (unit roundoff 2^-11),
# s = 2^-8, ref = rho for f and p / cs^2 for g.  Storing rounds the deviation
# delta_a = psi_a / w_a - ref to a relative 2^-11 of itself (deviations so
# small that d_a is subnormal carry an absolute error of at most 2^-25 s,
# negligible here), so the density sum_a psi_a moves by at most
# 2^-11 sum_a w_a |delta_a| <= 2^-11 max |delta|.  Each step stores once;
# streaming and the relaxation do not amplify the error, so after n steps it
# is at most n 2^-11 max |delta| (linear accumulation, the worst case), plus
# the FP32 arithmetic of the path.  The composition C = (rho - rho_v) /
# (rho_l - rho_v) carries the density error divided by rho_l - rho_v, the
# larger of the two relative errors (rho is measured relative to rho_l).
U16 = 2.0 ** -11
D2Q9_W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
D3Q19_W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def max_deviation(state, fields, lattice):
    """max over nodes and populations of |psi_a / w_a - ref| for an oracle
    state [2Q][N] and its fields (ref = rho for f, p / cs^2 for g)."""
    Q = lattice
    w = (D2Q9_W if Q == 9 else D3Q19_W)[:, None]
    df = np.abs(state[:Q] / w - fields["rho"][None, :]).max()
    dg = np.abs(state[Q:] / w - 3.0 * fields["p"][None, :]).max()
    return float(max(df, dg))


def fp16_storage_bound(max_dev, rho_l, rho_v, steps, fp32_part=2e-5):
    """Bound on the FP16-storage error of rho (relative to rho_l) and C
    after `steps` steps, given the largest deviation max |delta|."""
    return max(steps, 1) * U16 * max_dev / (rho_l - rho_v) + fp32_part


# The velocity with no floor.  u = (sum_a e_a g_a + dt/2 (S + rho g)) / rho,
# where the stored g deviations delta_a = g_a / w_a - p / cs^2 are of the
# size of the forcing terms while their first moment rho u is, for a resting
# drop, the small residual of a force balance.  A rounding to a relative eps
# of every deviation moves rho u by at most
# eps sum_a |e_a| w_a |delta_a| <= sqrt(d) eps max |delta|; a step rounds
# each deviation when it is stored and in the streaming sums, the solve and
# the collision, counted here as `ops` roundings of that size; over n steps
# the errors add at most linearly.  Relative to max |u|, with rho_v the
# smallest density:
#     n ops sqrt(d) eps max|delta| / (rho_v max|u|)
# plus the arithmetic of the velocity itself.
U32 = 2.0 ** -24
U64 = 2.0 ** -53


def velocity_bound(max_dev, rho_v, u_max, dim, steps, eps, ops=8, arith=2e-5):
    return max(steps, 1) * ops * np.sqrt(dim) * eps * max_dev / (rho_v * max(u_max, 1e-300)) + arith
