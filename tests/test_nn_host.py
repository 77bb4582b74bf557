"""Host build of the library's closest-point search (the target layout of
the set-up code and the octree search the kernels run): against brute force
over every target, the closest target's index must match exactly, ties
(duplicate targets, queries on grid points) going to the lowest user index,
cold, seeded by an arbitrary previous answer and by the closest target
itself or its neighbour in the sort order (the search then starts deep in
the octree), for 1 to 20,000 targets,
leaf occupancies 1 to 8 and forced depths 2 to 6, including a flat target
set (one axis of zero extent) and coordinates far from the origin."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r'''
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>
#include "amm_internal.h"
#include "amm_nn.h"
using namespace amm;
struct D4 { double x, y, z, w; };
struct F4 { float x, y, z, w; };
int main() {
    std::mt19937_64 g(3);
    std::uniform_real_distribution<double> u(-1, 1);
    int fails = 0;
    long long searches = 0;
    for (int M : {1, 3, 4, 5, 17, 64, 100, 1000, 4097, 20000}) {
        for (int variant = 0; variant < 9; ++variant) {
            // variants 0-3: occupancy rule with leaf 1, 2, 4, 8; 4-6: forced
            // depths 2, 4, 6; 7: flat set (z = 0); 8: offset far from the origin
            const int leaf = variant < 4 ? (1 << variant) : 8;
            const int depth = variant == 4 ? 2 : variant == 5 ? 4 : variant == 6 ? 6 : 0;
            const double off = variant == 8 ? 37.0 : 0.0;
            // a height field on a 1/16 grid: many exact duplicates
            std::vector<double> tgt(3 * (size_t)M);
            for (int i = 0; i < M; ++i) {
                tgt[3 * i] = std::round(u(g) * 16) / 16 + off;
                tgt[3 * i + 1] = std::round(u(g) * 16) / 16;
                tgt[3 * i + 2] = variant == 7 ? 0.0 : 0.25 * std::sin(3 * tgt[3 * i]);
            }
            TargetLayout tl;
            target_layout(tgt.data(), M, leaf, tl, depth);
            PairInfo pi{};
            pi.M = M;
            pi.grid_bits = tl.grid_bits;
            for (int c = 0; c < 3; ++c) {
                pi.glo[c] = tl.glo[c];
                pi.gscale[c] = tl.gscale[c];
                pi.cs[c] = tl.cs[c];
            }
            pi.gpad = tl.gpad;
            std::vector<D4> t4(M);
            for (int i = 0; i < M; ++i) t4[i] = {tl.tgt4[4 * i], tl.tgt4[4 * i + 1], tl.tgt4[4 * i + 2], tl.tgt4[4 * i + 3]};
            std::vector<F4> f4(M);
            for (int i = 0; i < M; ++i) f4[i] = {(float)t4[i].x, (float)t4[i].y, (float)t4[i].z, (float)t4[i].w};
            for (int q = 0; q < 300; ++q) {
                double qx, qy, qz;
                if (q % 4 == 0) {
                    const int k = (int)(g() % M);
                    qx = tgt[3 * k]; qy = tgt[3 * k + 1]; qz = tgt[3 * k + 2];
                } else {
                    qx = 1.5 * u(g) + off; qy = 1.5 * u(g); qz = 0.5 * u(g);
                }
                if (q % 7 == 0) { qx = std::round(qx * 32) / 32; qy = std::round(qy * 32) / 32; }
                const float fx = (float)qx, fy = (float)qy, fz = (float)qz;
                float fbd = INFINITY;
                int fbid = 0x7fffffff, fbpos = 0;
                for (int t = 0; t < M; ++t) {
                    const float d = sq3(f4[t].x - fx, f4[t].y - fy, f4[t].z - fz);
                    const int id = (int)f4[t].w;
                    if (d < fbd || (d == fbd && id < fbid)) { fbd = d; fbid = id; fbpos = t; }
                }
                double bd = INFINITY;
                int bid = 0x7fffffff, bpos = 0;
                for (int t = 0; t < M; ++t) {
                    const double d = sq3(t4[t].x - qx, t4[t].y - qy, t4[t].z - qz);
                    const int id = (int)t4[t].w;
                    if (d < bd || (d == bd && id < bid)) { bd = d; bid = id; bpos = t; }
                }
                // seeds: none, two random targets, the closest target itself
                // (the tightest bound: the search starts deepest), and a
                // target next to it in the sorted order
                for (int seed = -1; seed < 4; ++seed) {
                    int prev = seed < 0 ? -1 : (int)(g() % M);
                    if (seed == 2) prev = bpos;
                    if (seed == 3) prev = (bpos + 1) % M;
                    int pos;
                    double d2;
                    oct_search<double, D4>(pi, tl.cells.data(), tl.cells.data(), t4.data(), qx, qy, qz, prev, pos, d2);
                    ++searches;
                    if (d2 != bd || (int)t4[pos].w != bid) {
                        if (fails < 10)
                            std::printf("f64 M %d variant %d depth %d query %d seed %d: index %d d2 %.17g, brute force %d %.17g\n",
                                        M, variant, pi.grid_bits, q, prev, (int)t4[pos].w, d2, bid, bd);
                        ++fails;
                    }
                    float fd2;
                    if (seed == 2) prev = fbpos;
                    oct_search<float, F4>(pi, tl.cells.data(), tl.cells.data(), f4.data(), fx, fy, fz, prev, pos, fd2);
                    ++searches;
                    if (fd2 != fbd || (int)f4[pos].w != fbid) {
                        if (fails < 10)
                            std::printf("f32 M %d variant %d depth %d query %d seed %d: index %d d2 %.9g, brute force %d %.9g\n",
                                        M, variant, pi.grid_bits, q, prev, (int)f4[pos].w, fd2, fbid, fbd);
                        ++fails;
                    }
                }
            }
        }
    }
    // exact ties across cell boundaries: a lattice of targets, queries at the
    // midpoints between two lattice neighbours, each seeded with the tie
    // partner of the higher user index: the search must widen its start
    // box to the tie distance to find the lower index across the boundary
    for (int variant = 0; variant < 2; ++variant) {
        const int S = 12, M = S * S * S;
        std::vector<double> tgt(3 * (size_t)M);
        std::vector<int> perm(M);
        for (int i = 0; i < M; ++i) perm[i] = i;
        for (int i = M - 1; i > 0; --i) std::swap(perm[i], perm[(int)(g() % (i + 1))]);
        for (int i = 0; i < M; ++i) {
            const int c = perm[i];
            tgt[3 * i] = 0.125 * (c % S);
            tgt[3 * i + 1] = 0.125 * ((c / S) % S);
            tgt[3 * i + 2] = 0.125 * (c / (S * S));
        }
        TargetLayout tl;
        target_layout(tgt.data(), M, variant == 0 ? 1 : 2, tl);
        PairInfo pi{};
        pi.M = M;
        pi.grid_bits = tl.grid_bits;
        for (int c = 0; c < 3; ++c) {
            pi.glo[c] = tl.glo[c];
            pi.gscale[c] = tl.gscale[c];
            pi.cs[c] = tl.cs[c];
        }
        pi.gpad = tl.gpad;
        std::vector<F4> f4(M);
        std::vector<int> pos_of(M);
        for (int i = 0; i < M; ++i) {
            f4[i] = {(float)tl.tgt4[4 * i], (float)tl.tgt4[4 * i + 1], (float)tl.tgt4[4 * i + 2], (float)tl.tgt4[4 * i + 3]};
            pos_of[tl.tgt_user[i]] = i;
        }
        for (int a = 0; a < M; ++a)
            for (int ax = 0; ax < 3; ++ax) {
                double q[3] = {tgt[3 * a], tgt[3 * a + 1], tgt[3 * a + 2]};
                q[ax] += 0.0625;
                if (q[ax] > 0.125 * (S - 1)) continue;
                int b = -1;   // the lattice neighbour across the midpoint
                for (int t = 0; t < M; ++t)
                    if (tgt[3 * t + ax] == q[ax] + 0.0625 && tgt[3 * t + (ax + 1) % 3] == q[(ax + 1) % 3] &&
                        tgt[3 * t + (ax + 2) % 3] == q[(ax + 2) % 3]) b = t;
                const int lo_id = std::min(a, b), hi_id = std::max(a, b);
                int pos;
                float fd2;
                oct_search<float, F4>(pi, tl.cells.data(), tl.cells.data(), f4.data(), (float)q[0], (float)q[1],
                                      (float)q[2], pos_of[hi_id], pos, fd2);
                ++searches;
                if ((int)f4[pos].w != lo_id || fd2 != (float)(0.0625 * 0.0625)) {
                    if (fails < 10)
                        std::printf("lattice tie: query between %d and %d gave %d (%.9g)\n", lo_id, hi_id,
                                    (int)f4[pos].w, fd2);
                    ++fails;
                }
            }
    }
    std::printf("%d failures over %lld searches\n", fails, searches);
    return fails != 0;
}
'''


def test_octree_search_equals_brute_force(tmp_path):
    hipcc = shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)
    if hipcc is None:
        pytest.skip("no hipcc")
    src = tmp_path / "nn.hip"
    src.write_text(PROGRAM)
    exe = tmp_path / "nn"
    csrc = os.path.join(ROOT, "paper_2206_03410_amd", "csrc")
    subprocess.run([hipcc, "-std=c++17", "-O2", "--offload-host-only", "-I", csrc, "-I", os.path.join(ROOT, "include"),
                    "-x", "hip", str(src), os.path.join(csrc, "amm_setup.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout
