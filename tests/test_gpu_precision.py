"""Precision tier B: the coefficient-to-segment maps in bf16 on MFMA with
fp32 accumulation (forward: c and B rounded to bf16; adjoint: the backprojected
segment values Q_s and B rounded to bf16).

Parity: against the float64 oracle evaluated with the same rounding points.
Forward: relative L2 <= 1e-5 (both sides round the same float32 inputs c and
B; products of two bf16 values are exact in fp32, so only fp32 accumulation
separates them).  Adjoint: relative L2 <= 5e-5, because its rounding point Q
is an intermediate summed in fp32 over ~16 weighted residual terms per voxel
and projection: its error of ~sqrt(16) 2^-24 ~ 2.4e-7 relative makes a value
that close to a bf16 rounding boundary round the other way, with probability
p ~ 2 x 2.4e-7 / 2^-8 ~ 1.2e-4 per element, moving it by one bf16 unit (2^-8
relative); such flips add incoherently, giving ~sqrt(p) 2^-8 ~ 4e-5 relative
L2.  (Which Q values flip depends on the fp32 summation order, so no oracle
evaluated in float64 can take the same rounding decisions.)
The error against the unrounded float64 oracle is reported and bounded by the
bf16 unit roundoff scale (<= 1e-2).
"""
import numpy as np
import pytest
import torch

import oracle
from geoms import small, workload
from helpers import gpu_projector, rel_l2

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.tensor(np.asarray(a, dtype=np.float32), device=DEV)


def _geom(name):
    return {"small_l4": lambda: small(ell_max=4), "small_l8_seg16": lambda: small(ell_max=8, n_seg=16),
            "small_l6": lambda: small(ell_max=6), "c1": lambda: workload("c1"),
            "small_l10": lambda: small(ell_max=10), "small_l8_seg32": lambda: small(ell_max=8, n_seg=32)}[name]()


@pytest.mark.parametrize("name", ["small_l4", "small_l8_seg16", "small_l6", "c1", "small_l10", "small_l8_seg32"])
def test_bf16_forward(name):
    og = _geom(name)
    rng = np.random.default_rng(41)
    c = rng.standard_normal(og.vol_shape).astype(np.float32).astype(np.float64)
    U = oracle.unique_segments(og)
    Bq = oracle.bf16(og.B()[:, [cc % U for cc in range(og.n_seg)], :])
    ref_rounded = oracle.project(og, oracle.bf16(c), B=Bq)
    ref = oracle.project(og, c)
    P = gpu_projector(og, map_precision="bf16")
    got = P.forward(_t(c)).cpu().numpy()
    e_r, e = rel_l2(got, ref_rounded), rel_l2(got, ref)
    print(f"{name} bf16 forward: vs rounded oracle {e_r:.2e}, vs float64 oracle {e:.2e}")
    assert e_r <= 1e-5
    assert e <= 1e-2
    # the fp32 tier on the same projector object
    P.set_precision("fp32")
    assert rel_l2(P.forward(_t(c)).cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("name", ["small_l4", "small_l8_seg16", "small_l6", "c1", "small_l10", "small_l8_seg32"])
def test_bf16_adjoint(name):
    og = _geom(name)
    rng = np.random.default_rng(42)
    y = rng.standard_normal(og.data_shape).astype(np.float32).astype(np.float64)
    ref_rounded = oracle.adjoint_segment_first(og, y, round_q=oracle.bf16, round_b=oracle.bf16)
    ref = oracle.adjoint(og, y)
    P = gpu_projector(og, map_precision="bf16")
    got = P.adjoint(_t(y)).cpu().numpy()
    e_r, e = rel_l2(got, ref_rounded), rel_l2(got, ref)
    print(f"{name} bf16 adjoint: vs rounded oracle {e_r:.2e}, vs float64 oracle {e:.2e}")
    assert e_r <= 5e-5
    assert e <= 1e-2
