"""The compile-time 1D tables of the register-resident kernels (csrc/gauss_tables.h: Gauss points
written out from their closed forms, Lagrange values and derivatives from the product formula)
against the oracle's Gauss-Legendre rule and Lagrange basis, for Q1-Q4.  The header is compiled
as plain host C++; a wrong digit in a Gauss point or weight, or a slip in the product formula,
moves an entry far beyond the 1e-15 allowed."""
import os
import subprocess

import numpy as np
import pytest

from oracle import fe

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2005_00331_amd", "csrc")

PROGRAM = r"""
#define __host__
#define __device__
#include <cstdio>
#include "gauss_tables.h"
template <int K> void dump() {
  using T = mfpff::ConstTab<K>;
  for (int q = 0; q <= K; ++q) {
    std::printf("%d w %d %.17e\n", K, q, T::w(q));
    std::printf("%d x %d %.17e\n", K, q, T::x(q));
    for (int i = 0; i <= K; ++i) {
      std::printf("%d B %d %d %.17e\n", K, q, i, T::B(q, i));
      std::printf("%d D %d %d %.17e\n", K, q, i, T::D(q, i));
    }
  }
}
int main() { dump<1>(); dump<2>(); dump<3>(); dump<4>(); }
"""


@pytest.fixture(scope="module")
def tables(tmp_path_factory):
    d = tmp_path_factory.mktemp("tab")
    src, exe = d / "t.cpp", d / "t"
    src.write_text(PROGRAM)
    subprocess.run(["g++", "-std=c++17", "-O0", "-I", CSRC, str(src), "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    tab = {}
    for line in out.splitlines():
        parts = line.split()
        tab[tuple(parts[:-1])] = float(parts[-1])
    return tab


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_tables_match_the_oracle_basis(tables, k):
    xq, wq = fe.gauss_legendre_01(k + 1)
    B = fe.lagrange_values(k, xq)     # [q][i]
    Dd = fe.lagrange_derivs(k, xq)
    for q in range(k + 1):
        assert abs(tables[(str(k), "x", str(q))] - xq[q]) <= 1e-15
        assert abs(tables[(str(k), "w", str(q))] - wq[q]) <= 1e-15
        for i in range(k + 1):
            # the points agree to an ulp; the Lagrange products carry that through a few ulps
            assert abs(tables[(str(k), "B", str(q), str(i))] - B[q, i]) <= 4e-15 * max(1.0, abs(B[q, i]))
            # the derivative sums cancel terms up to ~16 in size: a few ulps of those
            assert abs(tables[(str(k), "D", str(q), str(i))] - Dd[q, i]) <= 1e-14 * max(1.0, abs(Dd[q, i]))
    assert abs(sum(tables[(str(k), "w", str(q))] for q in range(k + 1)) - 1.0) <= 1e-15


def test_even_degree_middle_point_is_a_node(tables):
    # at k = 2 and 4 the middle Gauss point is the middle node: a unit row of B and a zero
    # derivative of the middle basis function, exactly (the kernels drop those terms)
    for k in (2, 4):
        m = k // 2
        for i in range(k + 1):
            assert tables[(str(k), "B", str(m), str(i))] == (1.0 if i == m else 0.0)
        assert tables[(str(k), "D", str(m), str(m))] == 0.0
