"""The CPU oracle against its pins (no GPU). See tests/pins.py for what pins what."""
import os
import subprocess
import sys

import pytest

import oracle
import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(orc, pin):
    fails = pin(orc)
    assert not fails, "\n".join(fails[:10])


# Each entry plants one plausible mistake in oracle.c. Every one must trip a pin.
PLANTED = [
    ("light threshold read as strict", "return w > 0.0 && w <= delta;", "return w > 0.0 && w < delta;"),
    ("heavy threshold read as >=", "static int is_heavy(double w, double delta) { return w > delta; }",
     "static int is_heavy(double w, double delta) { return w >= delta; }"),
    ("fp32 sums kept in double", "float s = a + b;                   /* one binary32 rounding */",
     "double s = (double)a + (double)b;"),
    ("bucket upper bound off by one",
     "tb[v] = !isinf(t[v]) && ge_multiple(t[v], i, dl) && lt_multiple(t[v], i + 1.0, dl);",
     "tb[v] = !isinf(t[v]) && ge_multiple(t[v], i, dl) && lt_multiple(t[v], i + 2.0, dl);"),
    ("re-insertion mask taken after the min",
     "      for (int64_t v = 0; v < n; ++v)\n        tb[v] = !isinf(treq[v])",
     "      for (int64_t v = 0; v < n; ++v)\n        if (treq[v] < t[v]) t[v] = treq[v];\n"
     "      for (int64_t v = 0; v < n; ++v)\n        tb[v] = !isinf(treq[v])"),
    ("heavy phase masked by t_Bi instead of S",
     "      if (!S[u]) continue;\n      ssize++;\n      for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {\n"
     "        double we = weight_of(kind, w, e);\n        if (!is_heavy(we, dl)) continue;\n        if (tr) tr->heavy_relax++;\n"
     "        int ovf;\n        double c = plus(kind, t[u], we, &ovf);",
     "      if (!tb[u]) continue;\n      ssize++;\n      for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {\n"
     "        double we = weight_of(kind, w, e);\n        if (!is_heavy(we, dl)) continue;\n        if (tr) tr->heavy_relax++;\n"
     "        int ovf;\n        double c = plus(kind, t[u], we, &ovf);"),
    ("sign of the bucket-bound residual flipped", "static int ge_multiple(double t, double k, double delta) { return fma(-k, delta, t) >= 0.0; }",
     "static int ge_multiple(double t, double k, double delta) { return fma(k, delta, t) >= 0.0; }"),
    ("max-heap instead of min-heap", "if (h[p].key <= h[i].key) break;", "if (h[p].key >= h[i].key) break;"),
    ("certificate without the tightness walk", "if (!isinf(d[v]) && !seen[v]) { verdict = CERT_TIGHT; break; }",
     "if (0 && !isinf(d[v]) && !seen[v]) { verdict = CERT_TIGHT; break; }"),
    ("u32 overflow bound off by one", "if (s > U32_MAX_DIST) { *ovf = 1; return INFINITY; }",
     "if (s >= U32_MAX_DIST) { *ovf = 1; return INFINITY; }"),
    ("relax keeps the old bucket", "    bidx[v] = bucket_of(x, dl);\n    tent[v] = x;",
     "    if (bidx[v] < 0) bidx[v] = bucket_of(x, dl);\n    tent[v] = x;"),
    ("S accumulated from the next frontier",
     "      /* S = (S + tB) > 0 */\n      for (int64_t v = 0; v < n; ++v)\n        if (tb[v]) { S[v] = 1; trace_s_member(tr, v, (int64_t)i); }\n",
     ""),
    ("adjoint parent is the largest tight edge",
     "if (!ovf && c == d[v] && d[u] < d[v] && (pe[v] < 0 || e < pe[v])) { pe[v] = e; pv[v] = u; }",
     "if (!ovf && c == d[v] && d[u] < d[v] && (pe[v] < 0 || e > pe[v])) { pe[v] = e; pv[v] = u; }"),
    ("adjoint parent taken from an equal-distance vertex",
     "if (!ovf && c == d[v] && d[u] < d[v] && (pe[v] < 0 || e < pe[v])) { pe[v] = e; pv[v] = u; }",
     "if (!ovf && c == d[v] && (pe[v] < 0 || e < pe[v])) { pe[v] = e; pv[v] = u; }"),
    ("adjoint leaves absorbed vertices without a parent",
     "if (round_of[v] < 0) { round_of[v] = k; pe[v] = e; pv[v] = u; grew = 1; }", "if (0) {}"),
    ("adjoint drops the vertex's own coefficient", "for (int64_t v = 0; v < n; ++v) g[v] = (isinf(d[v]) || v == src) ? 0.0 : grad_dist[v];",
     "for (int64_t v = 0; v < n; ++v) g[v] = 0.0;"),
    ("adjoint does not pass subtree sums up", "        g[pv[v]] += g[v];\n", "\n"),
    ("edge source read as destination", "      int64_t v = col[e];\n      int ovf;\n      double c = plus(kind, d[u], weight_of(kind, w, e), &ovf);",
     "      int64_t v = u; (void)col;\n      int ovf;\n      double c = plus(kind, d[u], weight_of(kind, w, e), &ovf);"),
]


_RUN_PINS = """
import sys
sys.path[:0] = {paths!r}
import oracle, pins
o = oracle.Oracle({lib!r})
for pin in pins.ALL_PINS:
    try:
        f = pin(o)
    except Exception as exc:  # a crash or a refused status is a catch too
        f = [repr(exc)]
    if f:
        print("caught by", pin.__name__, f[0])
        sys.exit(1)
sys.exit(0)
"""


@pytest.mark.parametrize("name,old,new", PLANTED, ids=[p[0] for p in PLANTED])
def test_planted_mistake_is_caught(tmp_path, name, old, new):
    src = open(oracle.SOURCE).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {name}"
    path = tmp_path / "oracle_mut.c"
    path.write_text(src.replace(old, new, 1))
    lib = oracle.compile_source(str(path), str(tmp_path / "liboracle_mut.so"))
    here = os.path.dirname(os.path.abspath(__file__))
    code = _RUN_PINS.format(paths=[os.path.dirname(here), here], lib=lib)
    try:
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=20)
    except subprocess.TimeoutExpired:
        return  # the broken build never finishes a pin: caught
    assert r.returncode != 0, f"planted mistake '{name}' trips no pin\n{r.stdout}{r.stderr}"
