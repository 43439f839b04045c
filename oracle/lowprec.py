"""Emulation of the reduced-precision patch apply (Eq.(3) with the database
inverses and the restricted residuals rounded to FP32, BF16 or FP16).

The paper applies its patches in FP64 only; the reduced-precision variants are
an extension of this implementation.  The emulation fixes which values enter
the products, so that a device result can be judged against it:

* FP64 -> FP32 is round-to-nearest-even; FP32 -> BF16 and FP32 -> FP16 are
  round-to-nearest-even (two roundings, as a device converts FP64 data through
  FP32);
* FP16 uses power-of-two scales to stay inside its range: a database inverse
  X_j is multiplied by 2^-e_j and a restricted residual r_k by 2^-f_k before
  the FP16 rounding, where 2^-e maps the largest magnitude m (taken after the
  FP32 rounding) into [2^13, 2^14); the products are multiplied back by
  2^(e_j + f_k);
* BF16X3 splits each FP32-rounded operand into a BF16 high part and the BF16
  rounding of the remainder, and keeps the three leading products
  hi*hi + hi*lo + lo*hi (about 16 significant bits);
* the products of the rounded operands are summed exactly (float64 here); a
  device that sums them in FP32 stays within p_s * 2^-24 * sum|x||r| of this.

Test infrastructure only (see the package docstring).  Parity of the rounding
itself is pinned by exact bit patterns in the tests.
"""
from __future__ import annotations

import numpy as np


def round_fp32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def round_bf16(x32):
    """FP32 -> BF16 round-to-nearest-even, returned as float32 values."""
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    v = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    return v.view(np.float32)


def round_fp16(x32):
    return np.asarray(x32, dtype=np.float32).astype(np.float16).astype(np.float32)


def fp16_scale_exp(m32) -> int:
    """Exponent e with m * 2^-e in [2^13, 2^14) for a float32 magnitude m > 0;
    0 for m == 0."""
    m = float(m32)
    if m == 0.0:
        return 0
    _, E = np.frexp(np.float32(m))   # m = f 2^E, f in [0.5, 1)
    return int(E) - 14


def _round_operand(x, precision, scale_exp=0):
    x32 = round_fp32(x)
    if precision == "fp32":
        return x32.astype(np.float64)
    if precision == "bf16":
        return round_bf16(x32).astype(np.float64)
    if precision == "fp16":
        s = np.float32(2.0 ** (-scale_exp))
        return round_fp16(x32 * s).astype(np.float64)
    raise ValueError(precision)


def split_bf16(x):
    """High/low BF16 split of FP32-rounded values: hi = bf16(x32) and
    lo = bf16(x32 - hi) (the difference is exact in FP32)."""
    x32 = round_fp32(x)
    hi = round_bf16(x32)
    lo = round_bf16((x32 - hi).astype(np.float32))
    return hi.astype(np.float64), lo.astype(np.float64)


def rounded_database(X, precision):
    """Rounded database entries and their FP16 exponents (0 otherwise)."""
    out, exps = [], []
    for Xj in X:
        e = fp16_scale_exp(np.max(np.abs(round_fp32(Xj)))) if precision == "fp16" else 0
        out.append(split_bf16(Xj) if precision == "bf16x3" else _round_operand(Xj, precision, e))
        exps.append(e)
    return out, exps


def apply_lowprec(ptr, dofs, W, X, phi, r, omega=1.0, precision="bf16", return_bound=False):
    """Reduced-precision Eq.(3): z = omega W sum_k V_k^T (X~_phi(k) r~_k) with
    rounded operands; also returns, if asked, the per-dof bound
    omega W sum_k V_k^T (|X~| |r~|) used for FP32-accumulation tolerances."""
    Xr, ex = rounded_database(X, precision)
    r = np.asarray(r, dtype=np.float64)
    z = np.zeros_like(r)
    bnd = np.zeros_like(r)
    for k in range(len(ptr) - 1):
        d = dofs[ptr[k]:ptr[k + 1]]
        rk = r[d]
        j = phi[k]
        if precision == "bf16x3":
            # three leading products of the split operands: hi*hi + hi*lo + lo*hi
            (xh, xl), (rh, rl) = Xr[j], split_bf16(rk)
            np.add.at(z, d, xh @ rh + xh @ rl + xl @ rh)
            np.add.at(bnd, d, np.abs(xh) @ np.abs(rh) + np.abs(xh) @ np.abs(rl)
                      + np.abs(xl) @ np.abs(rh))
            continue
        f = fp16_scale_exp(np.max(np.abs(round_fp32(rk)))) if precision == "fp16" else 0
        rr = _round_operand(rk, precision, f)
        scale = 2.0 ** (ex[j] + f)
        np.add.at(z, d, (Xr[j] @ rr) * scale)
        np.add.at(bnd, d, (np.abs(Xr[j]) @ np.abs(rr)) * scale)
    z = omega * W * z
    if return_bound:
        return z, omega * W * bnd
    return z
