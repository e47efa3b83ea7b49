"""Algorithmic operation and byte counts of the hot path, used to place the
measured kernels on their rooflines.

Flops are the nominal count of a direct evaluation of the characteristic
interface flux (an FMA counts 2, add / mul / div / sqrt / max count 1, abs and
compares 0), per interface of one direction.  The kernels execute fewer where
an exact shortcut applies (TENO weights skipped when a bound proves that no
stencil is cut, the LLF halving folded into the projections), so a rate from
this count is an effective rate; the executed FP64 flops measured by the
hardware counters are reported next to it.

  per-point primitives (1/rho, |m|^2, p, a), amortised to one point  8 + 2 nd
  averaged (Roe) state, a, 1/a, b = (gamma-1)/a^2                   26 + 8 nt
  per stencil point (6): u_n, u.m, A = b(K rho - u.m + E),
      B = (u_n rho - m_n)/a, |u_n -+ a|, |u_n| maxima             6 (11 + 2 nt)
  maxima over the six points                                         10
  projections V = L U and g = L f (two acoustic fields 60 each,
      entropy 36, each shear field 18)                         120 + 36 + 18 nt
  LLF split of each field (6 points, both signs)                     31 nf
  reconstructions (2 per field)                          2 nf * (78 TENO5 | 72 WENO-Z5)
  back-projection F = R ghat                                         14 + 4 nt
  flux difference and residual update                                3 nc

with nt = nd - 1 tangents, nf = nc = nd + 2 fields.  3D TENO5: 1320 flops.
Compulsory HBM traffic of one RK substage: read U and dU, write U and dU,
4 * nc * 8 bytes per point (160 B in 3D, 128 B in 2D).
"""

PEAK_FP64_VALU_TFLOPS = 78.6
PEAK_FP32_VALU_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def flops_per_interface(nd: int, scheme: int) -> int:
    nt = nd - 1
    nc = nd + 2
    nf = nc
    recon = 78 if scheme == 1 else 72
    return ((8 + 2 * nd) + (26 + 8 * nt) + 6 * (11 + 2 * nt) + 10 + (120 + 36 + 18 * nt) + 31 * nf
            + 2 * nf * recon + (14 + 4 * nt) + 3 * nc)


def interfaces_per_sweep(n, nd: int, d: int) -> int:
    """Interfaces the algorithm evaluates in one sweep along direction d."""
    tot = int(n[d]) + 1
    for e in range(nd):
        if e != d:
            tot *= int(n[e])
    return tot


def compulsory_bytes_per_point(nd: int) -> int:
    return 4 * (nd + 2) * 8


def sweep_bytes_per_point(nd: int, first: bool) -> int:
    """Unavoidable HBM bytes of one convective sweep per point: read U, write
    the residual accumulator (first direction) or read and write it (later
    directions)."""
    nc = nd + 2
    return nc * 8 * (2 if first else 3)
