"""Host build of the coarse inverse's 4x4 pivot step (the preconditioner of
the Eq. 21 solve inverts each pivot block by its adjugate and tests it for
definiteness by Sylvester's criterion).  Checked on the CPU: inverses of
random symmetric positive definite blocks over a range of conditioning,
exact reciprocals of diagonal blocks, and rejection of indefinite and
singular blocks (the path that makes the kernel write an all-zero inverse)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r'''
#include <cmath>
#include <cstdio>
#include <random>
#include "amm_coarse_inv.h"

static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { ++fails; std::printf(__VA_ARGS__); std::printf("\n"); } } while (0)

int main() {
    std::mt19937_64 g(11);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    // random SPD blocks B B^T + eps I, eps from 1 down to 1e-6
    for (int it = 0; it < 4000; ++it) {
        const double eps = std::pow(10.0, -6.0 * (it % 7) / 6.0);
        double B[4][4], M[4][4], out[16];
        for (auto& r : B) for (auto& v : r) v = u(g);
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                double e = 0;
                for (int k = 0; k < 4; ++k) e += B[i][k] * B[j][k];
                M[i][j] = e + (i == j ? eps : 0.0);
            }
        const bool ok = amm::cinv_pivot_inverse(M, out);
        CHECK(ok, "SPD block rejected (eps %g)", eps);
        double res = 0, nrm = 0;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                double e = 0;
                for (int k = 0; k < 4; ++k) e += M[i][k] * out[4 * k + j];
                res = std::fmax(res, std::fabs(e - (i == j ? 1.0 : 0.0)));
                nrm = std::fmax(nrm, std::fabs(out[4 * i + j]));
                CHECK(out[4 * i + j] == out[4 * j + i], "inverse not symmetric");
            }
        // |M X - I| is bounded by the conditioning: cond(M) <= (|M| + eps) / eps with |M| <= 16
        CHECK(res <= 1e-13 * (16.0 + eps) / eps, "residual %g at eps %g", res, eps);
    }
    // diagonal blocks: the reciprocals, to a few ulps
    for (int it = 0; it < 1000; ++it) {
        double M[4][4] = {}, out[16];
        double d[4];
        for (int i = 0; i < 4; ++i) M[i][i] = d[i] = std::exp(6.0 * u(g));
        CHECK(amm::cinv_pivot_inverse(M, out), "diagonal block rejected");
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                const double want = i == j ? 1.0 / d[i] : 0.0;
                CHECK(std::fabs(out[4 * i + j] - want) <= 1e-15 * std::fabs(want), "diagonal %d %d", i, j);
            }
    }
    // indefinite: the first negative leading principal minor is the 1x1, the
    // 2x2, the 3x3 and the 4x4 one in turn
    const double cases[4][4][4] = {
        {{-1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}},
        {{1, 0, 0, 0}, {2, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}},
        {{1, 0, 0, 0}, {0, 1, 0, 0}, {2, 0, 1, 0}, {0, 0, 0, 1}},
        {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 3, 1}},
    };
    for (int c = 0; c < 4; ++c) {
        double M[4][4], out[16];
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) M[i][j] = i >= j ? cases[c][i][j] : cases[c][j][i];
        CHECK(!amm::cinv_pivot_inverse(M, out), "indefinite case %d accepted", c);
    }
    // singular: a zero row and column, and the zero block
    {
        double M[4][4] = {{2, 0, 0, 0}, {1, 2, 0, 0}, {0, 1, 2, 0}, {0, 0, 0, 0}}, out[16];
        CHECK(!amm::cinv_pivot_inverse(M, out), "singular block accepted");
        double Z[4][4] = {};
        CHECK(!amm::cinv_pivot_inverse(Z, out), "zero block accepted");
    }
    std::printf("%d failures\n", fails);
    return fails != 0;
}
'''


def test_pivot_inverse_host_build(tmp_path):
    hipcc = shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)
    if hipcc is None:
        pytest.skip("no hipcc")
    src = tmp_path / "pivot.hip"
    src.write_text(PROGRAM)
    exe = tmp_path / "pivot"
    csrc = os.path.join(ROOT, "paper_2206_03410_amd", "csrc")
    subprocess.run([hipcc, "-std=c++17", "-O2", "--offload-host-only", "-I", csrc, "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout
