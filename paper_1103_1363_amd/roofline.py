"""Algorithmic byte and flop accounting for the kernels of the solve path.

The paper's performance model (section 3) estimates a task's time as the
maximum over concurrent subtasks of latency + transferred bytes / bandwidth,
and its floating-point efficiency as the ratio of the ideal compute time to
that estimate.  The same accounting is used here to price every kernel
against the HBM roofline: only compulsory traffic counts (each link once per
half-lattice sweep, each input spinor once, each output once), never the
8-neighbour re-reads that caches absorb.

Units: one "site" is one output site of one parity; sizes in bytes.
"""
from __future__ import annotations

# Wilson hopping term per output site and right-hand side: 8 directions x
# (12 projection + 2 x 66 for two 3x3 complex mat-vecs + 24 accumulate)
# minus 24 for the first direction's accumulate.
DSLASH_FLOPS = 8 * (12 + 2 * 66 + 24) - 24
# two 6x6 Hermitian mat-vecs per site (clover apply): per block 30 complex
# off-diagonal products (6 flops), 6 real-diagonal products (2 flops) and
# 30 complex additions (2 flops)
CLOVER_FLOPS = 2 * (30 * 6 + 6 * 2 + 30 * 2)

PREC_BYTES = {"f64": 8, "f32": 4, "f16": 2}
# FP16 spinors carry one FP32 scale per site
PREC_NORM_BYTES = {"f64": 0, "f32": 0, "f16": 4}


def spinor_bytes(prec: str) -> int:
    """Bytes of one full spinor (12 complex) in storage precision prec."""
    return 24 * PREC_BYTES[prec] + PREC_NORM_BYTES[prec]


def link_bytes(prec: str, reals: int = 12) -> int:
    return reals * PREC_BYTES[prec]


def dslash_bytes(prec: str, nrhs: int = 1, link_reals: int = 12) -> int:
    """Compulsory bytes per output site of an even-odd hopping sweep.

    Eight links (four forward of this parity, four backward of the other),
    one input spinor and one output spinor per right-hand side.
    """
    return 8 * link_bytes(prec, link_reals) + nrhs * 2 * spinor_bytes(prec)


def full_lattice_dslash_bytes(prec: str, link_reals: int = 18) -> int:
    """Compulsory bytes per site of a full-lattice (not even-odd) sweep with
    perfect reuse: four links, one input and one output spinor."""
    return 4 * link_bytes(prec, link_reals) + 2 * spinor_bytes(prec)


def clover_bytes(prec: str) -> int:
    """72 reals of the two Hermitian 6x6 chiral blocks per site."""
    return 72 * PREC_BYTES[prec]


def fp_efficiency(flops: float, nbytes: float, bandwidth: float, peak_flops: float) -> float:
    """Model efficiency t_peak / t_exe with t_exe = max(t_mem, t_fp)."""
    t_fp = flops / peak_flops
    t_mem = nbytes / bandwidth
    return t_fp / max(t_fp, t_mem)


def sap_efficiency(eps_bs: float, t_fp: float, t_lm: float, t_tnw: float,
                   eps_lm: float = 0.8) -> float:
    """The paper's SAP preconditioner model (eq. sapmodel), with the block
    solver's own time T_bs (n+1)/n read as T_FP and its peak time as
    eps_bs * T_FP; times in any common unit."""
    return eps_bs * t_fp / max(t_fp + t_lm / eps_lm, t_tnw)


# MI355X published peaks
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6
FP32_VECTOR_TFLOPS = 157.3
BF16_MFMA_TFLOPS = 2500.0
FP16_MFMA_TFLOPS = 2500.0
