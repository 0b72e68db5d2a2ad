"""Planted mistakes in copies of the oracle must each fail at least one pin (CPU only).

Every mutant is one plausible slip -- a dropped term, a wrong sign or index, a flipped
comparison -- applied to a copy of the oracle source in a temporary directory.  The pinned
checks of tests/pins.py must notice every one of them.
"""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

import oracle

MUTANTS = {
    "hinge takes the highest part": ("} else if (k < hinge[e]) {", "} else if (k > hinge[e]) {"),
    "stale frontier entries not filtered": ("if (deg[v] != 1)\n                continue;", "if (0)\n                continue;"),
    "assignment sign flipped": ("(k + 6 - g[v1] - g[v2]) % 3", "(k + g[v1] + g[v2]) % 3"),
    "assignment reads the wrong vertex": ("uint32_t v2 = edges[3 * e + (k + 2) % 3];", "uint32_t v2 = edges[3 * e + (k + 1) % 3];"),
    "inclusive rank at lookup": ("uint64_t mask = below ? ((1ull << below) - 1) : 0;", "uint64_t mask = (1ull << below << 2) - 1;"),
    "range reduction by modulo": ("return (uint64_t)(((unsigned __int128)z * p) >> 64);", "return z % p;"),
    "seed added instead of xored": ("uint64_t s = keys[i] ^ seed;", "uint64_t s = keys[i] + seed;"),
    "stream offset dropped": ("uint64_t z0 = orc_fin(a + 1 * ORC_GAMMA);", "uint64_t z0 = orc_fin(a);"),
    "code packing stride": ("x |= (uint64_t)(codes8[v] & 3) << (2 * t);", "x |= (uint64_t)(codes8[v] & 3) << t;"),
    "non-zero pair count uses AND": ("uint64_t x = (w | (w >> 1)) & 0x5555555555555555ull;", "uint64_t x = (w & (w >> 1)) & 0x5555555555555555ull;"),
    "no push at degree 1": ("if (deg[u] == 1)\n                    next[nn++] = u;", "if (deg[u] == 0)\n                    next[nn++] = u;"),
    "unstable counting sort": ("order[start[slot]++] = (uint32_t)e;", "order[--start[slot + 1]] = (uint32_t)e;"),
    "label is the vertex, not the edge": ("lab[v] ^= (uint32_t)e;", "lab[v] ^= v;"),
    "digest length fold dropped": ("*a_out = orc_fin(A ^ sa ^ len);", "*a_out = orc_fin(A ^ sa);"),
    "digest position salt dropped": ("B += orc_fin(w ^ (sb + j * ORC_GAMMA));", "B += orc_fin(w ^ sb);"),
    "digest reads past the key": ("if (p < len)\n                w |= ", "if (1)\n                w |= "),
    "degree limit off by one": ("if (maxdeg > ORC_MAX_DEGREE) {", "if (maxdeg >= ORC_MAX_DEGREE) {"),
    "duplicates reported as core": ("status = ORC_EDUP;", "status = ORC_ECORE;"),
    "part size rounds down": ("return (uint64_t)((num + den - 1) / den);", "return (uint64_t)(num / den);"),
    "rank counts only g = 0": ("count += codes8[v] != 0;", "count += codes8[v] == 3;"),
    "static function sign flipped": ("(values[e] + 2 * sigma - u[va] - u[vb]) % sigma", "(values[e] + u[va] + u[vb]) % sigma"),
    "static function field one bit short": ("while (b < 64 && ((sigma - 1) >> b) != 0)", "while (b < 64 && ((sigma - 1) >> (b + 1)) != 0)"),
    "static function packing shifted": ("|= (uint64_t)((u[v] >> t) & 1u) << (bit % 64);", "|= (uint64_t)((u[v] >> t) & 1u) << ((bit + 1) % 64);"),
    "static function lookup drops a vertex": ("+ orc_sf_field(words, b, t[2])) % sigma", ") % sigma"),
    "ranked lookup counts the vertex itself": ("for (uint64_t x = v - v % ORC_SFR_BLOCK; x < v; x++)",
                                               "for (uint64_t x = v - v % ORC_SFR_BLOCK; x <= v; x++)"),
    "ranked layout keeps zero fields": ("if (orc_sf_field(words, b, v) != 0) {", "if (1) {"),
    "ranked field index skips one": ("orc_put_field(vals, b, i++, ", "orc_put_field(vals, b, ++i, "),
    "ranked lookup reads the next block's sample": ("uint64_t r = rank[v / ORC_SFR_BLOCK];",
                                                    "uint64_t r = rank[v / ORC_SFR_BLOCK + 1];"),
    "hem signature adds the seed": ("return orc_fin((key ^ seed) + 4 * ORC_GAMMA);", "return orc_fin((key + seed) + 4 * ORC_GAMMA);"),
    "hem bucket key not swapped": ("return (sig << 32) | (sig >> 32);", "return sig;"),
    "hem bucket offset dropped": ("return bucket_off[b] + orc_eval_edge(", "return 0 * bucket_off[b] + orc_eval_edge("),
    "hem string signature folded to its first word": ("*y = sigs2 ? sigs2[i] : *x;", "*y = *x;"),
    "hem pair hash without the seed on the second word": ("orc_edge_of_digest(x[i] ^ seed, y[i] ^ seed, P, edges + 3 * i);",
                                                         "orc_edge_of_digest(x[i] ^ seed, y[i], P, edges + 3 * i);"),
    "hem string bucket key unswapped": ("*x = orc_hem_bucket_key(sigs[i]);", "*x = sigs2 ? sigs[i] : orc_hem_bucket_key(sigs[i]);"),
    "hem bucket from the low bits": ("uint64_t b = k ? sig >> (64 - k) : 0;", "uint64_t b = k ? sig & ((1ull << k) - 1) : 0;"),
    "general r hinge takes the higher position": ("} else if (hinge[e] > k) {", "} else if (hinge[e] < k) {"),
    "general r deletes skip the last vertex": ("            for (uint32_t k = 0; k < r; k++) {\n                uint32_t u = edges[(uint64_t)r * e + k];",
                                               "            for (uint32_t k = 0; k + 1 < r; k++) {\n                uint32_t u = edges[(uint64_t)r * e + k];"),
    "general r edges read with stride 3": ("            uint32_t v = edges[(uint64_t)r * e + k];", "            uint32_t v = edges[(uint64_t)3 * e + k];"),
}


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="mphx_mutants_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(workdir, name):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {old!r}"
    tag = "".join(ch if ch.isalnum() else "_" for ch in name)
    path = os.path.join(workdir, tag + ".c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    so = oracle.compile_oracle(path, os.path.join(workdir, tag + ".so"), extra=("-w",))
    # A planted mistake may index out of bounds and crash: run the pins in a child process;
    # a crash counts as caught.
    code = (
        "import sys, oracle, pins\n"
        f"bad = pins.run_all(oracle.Oracle(oracle.load({so!r})))\n"
        "print('\\n'.join(bad[:5]))\n"
        "sys.exit(3 if bad else 0)\n"
    )
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, PYTHONPATH=os.pathsep.join([root, os.path.join(root, "tests")]))
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode != 0, f"planted mistake '{name}' passed every pin"
