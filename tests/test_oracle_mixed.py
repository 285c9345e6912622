"""Pins of the oracle's mixed-precision emulation (oracle/mixed.py), no GPU.

  * bfloat16 rounding: hand-computed bit patterns (ties to even, carry into
    the exponent, overflow to infinity, subnormals, signed zero, NaN), and the
    same results as torch's float32 -> bfloat16 conversion (a library routine)
    on random values and on every tie of a range of exponents; a truncating
    conversion (a plausible mistake) fails the tie pins;
  * the FP32 cycle stays within a few units of float32 round-off of the FP64
    oracle (and is not the FP64 cycle); BF16 storage moves it by about the
    bfloat16 unit round-off, and with no BF16 levels it is the FP32 cycle;
  * the refinement-form solver with FP32 cycles needs the FP64 stationary
    iteration's cycle counts (equal in exact arithmetic: the cycle is affine,
    Sec. 1) within one, and its FP64 residual meets the tolerance."""
import numpy as np
import pytest
import torch

from mginputs import configs as C, hierarchy as H
from oracle import lmg as O
from oracle import mixed as M


def _bits(x):
    return [int(v) >> 16 for v in M.bf16_round(np.array(x, dtype=np.float32)).view(np.uint32)]


def test_bf16_hand_computed_bit_patterns():
    one_ulp = 2.0 ** -7          # bfloat16 spacing just above 1
    cases = [
        (1.0, 0x3F80),
        (1.0 + one_ulp, 0x3F81),                      # exactly representable
        (1.0 + one_ulp / 2, 0x3F80),                  # tie, 0x3F80 is even: down
        (1.0 + 3 * one_ulp / 2, 0x3F82),              # tie, 0x3F81 is odd: up
        (1.0 + one_ulp / 2 + 2.0 ** -20, 0x3F81),     # just above the tie: up
        (-(1.0 + one_ulp / 2 + 2.0 ** -20), 0xBF81),
        (2.0 - one_ulp / 2, 0x4000),                  # tie at 0x3FFF (odd): carry into the exponent
        (3.3895313892515355e38, 0x7F7F),              # largest finite bfloat16
        (3.4e38, 0x7F80),                             # rounds past it: infinity
        (np.inf, 0x7F80), (-np.inf, 0xFF80),
        (0.0, 0x0000), (-0.0, 0x8000),
        (9.183549615799121e-41, 0x0001),              # smallest bfloat16 subnormal
    ]
    got = _bits([c[0] for c in cases])
    assert got == [c[1] for c in cases], [hex(g) for g in got]
    nan = M.bf16_round(np.array([np.nan], dtype=np.float32))
    assert np.isnan(nan[0]) and (int(nan.view(np.uint32)[0]) & 0x00400000)


def _torch_bf16(x):
    return torch.tensor(x).to(torch.bfloat16).to(torch.float32).numpy()


def test_bf16_matches_library_conversion():
    g = C.rng(9, 1, 0)
    x = np.concatenate([g.standard_normal(20000) * 10.0 ** g.uniform(-30, 30, 20000),
                        g.uniform(-1e-38, 1e-38, 2000)]).astype(np.float32)
    # every tie (low 16 bits 0x8000) for a range of kept patterns
    kept = np.arange(0x3E00, 0x4200, dtype=np.uint32)
    ties = ((kept << 16) | 0x8000).view(np.float32)
    for v in (x, ties, -ties):
        assert np.array_equal(M.bf16_round(v).view(np.uint32), _torch_bf16(v).view(np.uint32))


def test_bf16_truncation_mistake_fails_the_tie_pins():
    def truncate(v):
        return (np.asarray(v, dtype=np.float32).view(np.uint32) & 0xFFFF0000).view(np.float32)
    v = np.array([1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20], dtype=np.float32)
    assert not np.array_equal(truncate(v), _torch_bf16(v))
    assert np.array_equal(M.bf16_round(v), _torch_bf16(v))


def _problem(side=65, B=4):
    w = C.block_diffusion(2, side, -2, 2, B=B, K=3)
    J = w.hier.nlevels
    flat = C.random_params(J, 3, 3, 3, seed=11, spread=0.1)
    lv = O.make_levels(w.hier.A, w.hier.P, w.hier.R)
    return w, lv, O.unpack(flat, J, 3, 3, 3)


def _err(a, b):
    return float((np.abs(a - b).max(axis=0) / np.abs(b).max(axis=0)).max())


def test_fp32_and_bf16_cycles_against_fp64():
    w, lv, prm = _problem()
    lv32 = M.make_levels32(lv)
    f = w.f
    e64 = O.lmg(lv, prm, 0, f, np.zeros_like(f))
    e32 = M.lmg32(lv32, prm, 0, f.astype(np.float32), None)
    e16 = M.lmg32(lv32, prm, 0, f.astype(np.float32), None, bf16_levels={0, 1})
    e16_none = M.lmg32(lv32, prm, 0, f.astype(np.float32), None, bf16_levels=())
    assert e32.dtype == np.float32 and e16.dtype == np.float32
    err32, err16 = _err(e32, e64), _err(e16, e64)
    print(f"fp32 {err32:.2e} bf16 {err16:.2e}")
    # about 100 dependent float32 roundings per V(2,2) cycle: a few 1e-6 at most; not the FP64 cycle
    assert 1e-9 < err32 <= 2e-6
    # bfloat16 unit round-off 2^-9 ~ 2e-3 on each stored intermediate
    assert 1e-4 < err16 <= 2e-2
    assert np.array_equal(e16_none, e32)
    # a cycle from a nonzero iterate: the same bound
    u = C.rng(9, 2, 0).standard_normal(f.shape)
    assert _err(M.lmg32(lv32, prm, 0, f.astype(np.float32), u.astype(np.float32)), O.lmg(lv, prm, 0, f, u)) <= 2e-6


def test_fp32_refinement_needs_the_fp64_cycle_counts():
    w, lv, prm = _problem(B=3)
    ref = O.solve(lv, prm, w.f, rtol=1e-8)
    mix = M.solve_mixed(lv, prm, w.f, rtol=1e-8)
    rel = np.linalg.norm(w.f - w.hier.A[0] @ mix.u, axis=0) / np.linalg.norm(w.f, axis=0)
    print("fp64", ref.iters, "fp32 refinement", mix.iters)
    assert np.all(rel <= 1e-8) and np.all(mix.converged)
    assert np.all(np.abs(mix.iters - ref.iters) <= 1)
    # BF16 storage slows the iteration down, never below the FP32 counts by more than one
    b16 = M.solve_mixed(lv, prm, w.f, rtol=1e-8, bf16_levels={0, 1})
    print("bf16 refinement", b16.iters)
    assert np.all(b16.converged) and np.all(b16.iters >= mix.iters - 1)
