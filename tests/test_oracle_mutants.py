"""The oracle's tree pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's source (on the CPU,
in a temporary directory), builds it, and runs the pin that is meant to
catch it: the pin must fail.  The oracle itself is untouched; the tree pins
(tests/test_oracle_tree_pins.py) pass on it.
"""
import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

import oracle
from tests import test_oracle_cic_amr as C
from tests import test_oracle_dipic as DI
from tests import test_oracle_octree as O3
from tests import test_oracle_tree_pins as P

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.cpp")

# name: (exact text in oracle.cpp, replacement, the pin that must fail)
MUTANTS = {
    "face coefficient uses the larger cell": (
        "double c = std::min(ha, hb) / ((ha + hb) / 2.0);",
        "double c = std::max(ha, hb) / ((ha + hb) / 2.0);",
        lambda L: P.check_fv_coarse_fine_faces(0, L)),
    "coarsen when a child holds exactly n_lo": (
        "if (!(smax <= n_hi && cmin < n_lo)) continue;",
        "if (!(smax <= n_hi && cmin <= n_lo)) continue;",
        P.check_coarsen_rule),
    "coarsen sums the species": (
        "smax = std::max(smax, s);",
        "smax = smax + s;",
        P.check_coarsen_rule),
    "coarsen ignores finer touching leaves": (
        "if (!inside && b->level > P->level + 1) { ok = false; break; }",
        "if (!inside && b->level > P->level + 2) { ok = false; break; }",
        P.check_coarsen_rule),
    "node potential over four leaves always": (
        "val = s / (double)kv.second.size();",
        "val = s / 4.0;",
        lambda L: P.check_hanging_nodes(False, L)),
    "merge ignores the velocity octant": (
        "if (ox != oy) return ox < oy;",
        "(void)ox; (void)oy;",
        P.check_merge_pairs),
    "cloud reaches to the wrong side": (
        "const int64_t Xn = X + (gx >= (T)0 ? (int64_t)S : -(int64_t)S);",
        "const int64_t Xn = X + (gx >= (T)0 ? -(int64_t)S : (int64_t)S);",
        lambda L: C.check_area_overlaps(1, L)),
    "ghost over finer leaves shared equally whatever their size": (
        "const uint64_t part = units >> (2 * dl[k]);",
        "const uint64_t part = units / dl.size();",
        lambda L: C.check_area_overlaps(1, L)),
    "merge breaks ties by the larger id": (
        "return P[x].id < P[y].id;",
        "return P[x].id > P[y].id;",
        P.check_merge_pairs),
    "trilinear weight takes the wrong side in z": (
        "const T wz = (c >> 2) ? f[2] : (T)1 - f[2];",
        "const T wz = (c >> 2) ? (T)1 - f[2] : f[2];",
        O3.check_trilinear),
    "octree balance allows two levels": (
        "if (b->level > a->level + 1) { mark.push_back(a); break; }\n      }\n      for (ONode* a : mark)",
        "if (b->level > a->level + 2) { mark.push_back(a); break; }\n      }\n      for (ONode* a : mark)",
        O3.check_mesh),
    "octree locate sends points on a mid-plane down": (
        "if (s[a] >= (2 * n->i[a] + 1) * hh) c |= 1 << a;",
        "if (s[a] > (2 * n->i[a] + 1) * hh) c |= 1 << a;",
        O3.check_locate),
    "ball refinement stops a level early": (
        "if (n->level >= d.disk_level || n->level >= d.max_level) continue;\n          double r2",
        "if (n->level + 1 >= d.disk_level || n->level >= d.max_level) continue;\n          double r2",
        O3.check_mesh),
    "implicit susceptibility without the half": (
        "return (((s.charge / s.mass) * ((d.dt * d.dt) * 0.5))",
        "return (((s.charge / s.mass) * ((d.dt * d.dt) * 1.0))",
        lambda L: DI.check_cold_plasma(L, wdts=(4.0,))),
    "filtered acceleration not averaged": (
        "q.b = (q.b + dv) * (T)0.5;",
        "q.b = dv;",
        lambda L: DI.check_cold_plasma(L, wdts=(1.5,))),
    "implicit Thomas elimination with the wrong sign": (
        "dp[i] = (r - a * dp[i - 1]) / m;",
        "dp[i] = (r + a * dp[i - 1]) / m;",
        DI.check_implicit_solve),
    "wall susceptibility over a whole cell": (
        "chi[i] = (i == 0 || i == N) ? 2.0 * c : c;",
        "chi[i] = c;",
        DI.check_implicit_solve),
    "octree nodal E divides by eight always": (
        "const double e = sum[a] / (double)k;",
        "const double e = sum[a] / 8.0;",
        O3.check_nodal_e),
}


@pytest.fixture(scope="module")
def mutant_libs():
    src = open(SRC).read()
    tmp = tempfile.mkdtemp(prefix="oracle_mutants_")
    hdr = os.path.join(os.path.dirname(SRC), "oracle.h")

    def build(item):
        k, (name, (old, new, _)) = item
        assert src.count(old) == 1, f"mutation site of '{name}' not found once"
        d = os.path.join(tmp, str(k))
        os.makedirs(d)
        with open(os.path.join(d, "oracle.cpp"), "w") as f:
            f.write(src.replace(old, new))
        subprocess.check_call(["cp", hdr, d])
        lib = os.path.join(d, "liboracle.so")
        subprocess.check_call(["g++", "-O1", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", lib, os.path.join(d, "oracle.cpp")])
        return name, lib
    with ThreadPoolExecutor(max_workers=4) as ex:
        built = dict(ex.map(build, enumerate(MUTANTS.items())))
    return {name: oracle.load_lib(path) for name, path in built.items()}


@pytest.mark.parametrize("name", list(MUTANTS))
def test_pin_catches_planted_mistake(name, mutant_libs):
    check = MUTANTS[name][2]
    with pytest.raises(AssertionError):
        check(mutant_libs[name])
