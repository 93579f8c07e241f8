"""Each plausible mistake planted in a copy of the oracle (a wrong meet, a
dropped kill or gen term, a swapped space test, a lost loop-entry rule, ...)
must be caught by at least one of the pins.  Runs on the CPU with gcc."""
import glob
import os
import subprocess

import numpy as np
import pytest

import checkers
import oracle
import synth
from test_oracle_pins import GOLDEN, PLACEMENTS, VK, bits_of, check_expect, load_golden
from test_oracle_placements import loopy, rows, value_read

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "ave_meet_or": ("meet &= out[s][ix(g, g->pi[k], w)];", "meet |= out[s][ix(g, g->pi[k], w)];"),
    "nu_no_kill": ("v = use_s(g, s, b, w) | (out & ~g->W[ix(g, b, w)]);", "v = use_s(g, s, b, w) | out;"),
    "ave_no_nu_gen": ("vin = nu[s][ix(g, q, w)] | meet;", "vin = meet;"),
    "transfer_space_swapped": ("uint64_t a1 = ((int)g->space[b] == s) ? (in_s | Wb) : (in_s & ~Wb);",
                               "uint64_t a1 = ((int)g->space[b] != s) ? (in_s | Wb) : (in_s & ~Wb);"),
    "transfer_no_stale": ("uint64_t a1 = ((int)g->space[b] == s) ? (in_s | Wb) : (in_s & ~Wb);",
                          "uint64_t a1 = ((int)g->space[b] == s) ? (in_s | Wb) : in_s;"),
    "later_no_neutral": ("all &= (lp | np);", "all &= lp;"),
    "later_no_any": ("uint64_t vin = all & any & vmask(g, w);", "uint64_t vin = all & vmask(g, w);"),
    "ins_edge_no_le": ("later_e & (le_mask(&g, e) | ~lin[s][ix(&g, q, w)]) & vmask(&g, w);",
                       "later_e & (~lin[s][ix(&g, q, w)]) & vmask(&g, w);"),
    "mayp_no_le": ("min |= (eag(g, nu[s], aveout[s], p, q, w) | mout[s][ix(g, p, w)]) & ~le_mask(g, e);",
                   "min |= (eag(g, nu[s], aveout[s], p, q, w) | mout[s][ix(g, p, w)]);"),
    "later_no_stop": ("uint64_t vout = vin & ~use_stop(g, s, q, w) & ~wr_s(g, s, q, w);",
                      "uint64_t vout = vin & ~wr_s(g, s, q, w);"),
    "avf_no_entry_gen": ("vin = ins_entry[s][ix(g, q, w)] | meet;", "vin = meet;"),
    "fv_wrong_space": ("uint64_t np = (fv(g, s, nu, aveout, mout, p, q, e, w) & fv(g, o, nu, aveout, mout, p, q, e, w)) |",
                       "uint64_t np = (fv(g, s, nu, aveout, mout, p, q, e, w) & fv(g, s, nu, aveout, mout, p, q, e, w)) |"),
    "after_dev_from_host": ("for (int b = 0; b < nb; ++b) if (space[b] == 1) { after_dev[b] = 1; stk[top++] = b; }",
                            "for (int b = 0; b < nb; ++b) if (space[b] == 0) { after_dev[b] = 1; stk[top++] = b; }"),
    "map_from_wrong_end": ("if ((ins_edge_h[(size_t)e * g.wd + w] & bit) && !before_dev[t]) from = 1;",
                           "if ((ins_edge_h[(size_t)e * g.wd + w] & bit) && !before_dev[q]) from = 1;"),
    "alloc_always": ("((dev_access && !to && !from) ? 4 : 0)", "(dev_access ? 4 : 0)"),
    "exit_not_live": ("if (b == g->exit) return g->lx[s][w];", "if (b == g->exit) return 0;"),
    # firstprivate
    "fp_read_is_device_use": ("if (g->space[b] == 1) return s == 1 ? (r & ~g->fp[w]) : (r & g->fp[w]);",
                              "if (g->space[b] == 1) return s == 1 ? r : 0ull;"),
    "fp_no_host_use": ("if (g->space[b] == 1) return s == 1 ? (r & ~g->fp[w]) : (r & g->fp[w]);",
                       "if (g->space[b] == 1) return s == 1 ? (r & ~g->fp[w]) : 0ull;"),
    "fp_no_kill": ("if (s == 1 && g->space[b] == 1) a1 &= ~(g->R[ix(g, b, w)] & g->fp[w]);", ""),
    "fp_device_written": ("g.fp[w] = scalar[w] & ~dev_w & vmask(&g, w);", "g.fp[w] = scalar[w] & vmask(&g, w);"),
    "fp_clause_on_host": ("fp_clause[ix(&g, b, w)] = space[b] == 1 ? (R[ix(&g, b, w)] & g.fp[w]) : 0ull;",
                          "fp_clause[ix(&g, b, w)] = R[ix(&g, b, w)] & g.fp[w];"),
    # loop-entry refinement
    "live_edge_copy_not_a_read": ("lo |= (li[s][ix(g, g->si[e], w)] & ~ig[s][(size_t)e * g->wd + w]) | ig[o][(size_t)e * g->wd + w];",
                                  "lo |= (li[s][ix(g, g->si[e], w)] & ~ig[s][(size_t)e * g->wd + w]);"),
    "live_entry_copy_not_a_read": ("uint64_t v = ((a & ~ie[s][ix(g, q, w)]) | ie[o][ix(g, q, w)]) & vmask(g, w);",
                                   "uint64_t v = (a & ~ie[s][ix(g, q, w)]) & vmask(g, w);"),
    "live_edge_copy_no_replace": ("lo |= (li[s][ix(g, g->si[e], w)] & ~ig[s][(size_t)e * g->wd + w]) | ig[o][(size_t)e * g->wd + w];",
                                  "lo |= li[s][ix(g, g->si[e], w)] | ig[o][(size_t)e * g->wd + w];"),
    "live_entry_copy_no_replace": ("uint64_t v = ((a & ~ie[s][ix(g, q, w)]) | ie[o][ix(g, q, w)]) & vmask(g, w);",
                                   "uint64_t v = (a | ie[o][ix(g, q, w)]) & vmask(g, w);"),
    "live_no_kill": ("uint64_t a = rd | (lo & ~kill);", "uint64_t a = rd | lo;"),
    "live_other_space_read": ("uint64_t rd = is_call(g, q) ? ~0ull : use_s(g, s, q, w);",
                              "uint64_t rd = is_call(g, q) ? ~0ull : use_s(g, o, q, w);"),
    "refine_every_edge": ("if (kind[e] != KIND_LOOP_ENTRY) continue;", ""),
    "refine_wrong_space": ("ig[s][(size_t)e * g.wd + w] &= li[s][ix(&g, t, w)];",
                           "ig[s][(size_t)e * g.wd + w] &= li[1 - s][ix(&g, t, w)];"),
    # pure lazy
    "lazy_ignored": ("return (!g->lazy && g->kind[e] == KIND_LOOP_ENTRY) ? ~0ull : 0ull;",
                     "return (g->kind[e] == KIND_LOOP_ENTRY) ? ~0ull : 0ull;"),
    "lazy_mayp_still_stops": ("min |= (eag(g, nu[s], aveout[s], p, q, w) | mout[s][ix(g, p, w)]) & ~le_mask(g, e);",
                              "min |= (eag(g, nu[s], aveout[s], p, q, w) | mout[s][ix(g, p, w)]) & ~(g->kind[e] == KIND_LOOP_ENTRY ? ~0ull : 0ull);"),
    "fp_alloc_too": ("if (space[q] == 1 && (((R[ix(&g, q, w)] & ~g.fp[w]) | W[ix(&g, q, w)]) & bit)) dev_access = 1;",
                     "if (space[q] == 1 && ((R[ix(&g, q, w)] | W[ix(&g, q, w)]) & bit)) dev_access = 1;"),
}


def run_variant_pins():
    """The placement variants: hand-derived worked examples, the refinement against the
    path search, the pure lazy variant against relabelled loop entries."""
    for path in sorted(glob.glob(os.path.join(GOLDEN, "P*.json"))):
        g, cfg, pos = load_golden(path)
        for name, exp in g.get("variants", {}).items():
            try:
                check_expect(g, cfg, pos, oracle.solve(cfg, placement=PLACEMENTS[name]), exp)
            except AssertionError:
                return False
    for seed in range(12):
        cfg = loopy(seed, marks=seed % 2 == 1)
        base = oracle.solve(cfg)
        ref = oracle.solve(cfg, placement=oracle.PLACEMENT_REFINE)
        V = checkers.View(cfg)
        ie0, ig0 = rows(base, cfg.wd)
        ie1, ig1 = rows(ref, cfg.wd)
        if ie1 != ie0:
            return False
        for p in range(cfg.n_blocks):
            for (t, e) in V.succ[p]:
                for s in (0, 1):
                    if int(cfg.edge_kind[e]) != 2:
                        if ig1[s][e] != ig0[s][e]:
                            return False
                        continue
                    for v in range(cfg.n_vars):
                        if (ig0[s][e] >> v) & 1:
                            if bool((ig1[s][e] >> v) & 1) != value_read(V, ie0, ig0, s, t, v):
                                return False
                        elif (ig1[s][e] >> v) & 1:
                            return False
        if checkers.check_invariants(cfg, ref):
            return False
        lazy = oracle.solve(cfg, placement=oracle.PLACEMENT_LAZY)
        plain = synth.CFG(**{f: getattr(cfg, f) for f in cfg.__dataclass_fields__})
        plain.edge_kind = np.where(np.asarray(cfg.edge_kind) == 2, 0, np.asarray(cfg.edge_kind)).astype(np.uint8)
        d = oracle.solve(plain)
        if any(not np.array_equal(lazy[k], d[k]) for k in d):
            return False
        if checkers.check_invariants(cfg, lazy):
            return False
    return True


def run_pins():
    """A compact version of the pin suite; returns True if every pin holds."""
    try:
        if not run_variant_pins():
            return False
        for path in sorted(glob.glob(os.path.join(GOLDEN, "P*.json"))):
            g, cfg, pos = load_golden(path)
            r = oracle.solve(cfg)
            exp = g["expect"]
            inv = {int(pos[i]): i for i in range(len(pos))}
            for k in ("nu_h", "nu_d", "ave_h", "ave_d", "avf_h", "avf_d"):
                if k in exp and bits_of(r[k]) != exp[k]:
                    return False
            for k in ("ins_edge_h", "ins_edge_d"):
                if sorted(inv[e] for e in range(cfg.n_edges) if int(r[k][e, 0]) & 1) != sorted(exp[k]):
                    return False
            for k in ("ins_entry_h", "ins_entry_d"):
                if [b for b in range(cfg.n_blocks) if int(r[k][b, 0]) & 1] != sorted(exp[k]):
                    return False
            if [int(x) for x in r["var_kind"]] != [VK[x] for x in exp["var_kind"]]:
                return False
            for k, want in g.get("expect_words", {}).items():
                if [int(x) for x in r[k][:, 0]] != want:
                    return False
        for seed in range(8):
            cfg = synth.random_dag(seed, 9, 65, p_loop_entry=0.3 if seed % 2 else 0.0)
            r = oracle.solve(cfg)
            nu_h, nu_d = checkers.mop_nu(cfg)
            if checkers.rows_int(r["nu_h"]) != nu_h or checkers.rows_int(r["nu_d"]) != nu_d:
                return False
            ave = checkers.mop_valid(cfg, [nu_h, nu_d], [{}, {}])
            if (checkers.rows_int(r["ave_h"]), checkers.rows_int(r["ave_d"])) != ave:
                return False
            after, before = checkers.reach_labels(cfg)
            if r["after_dev"].tolist() != after.tolist() or r["before_dev"].tolist() != before.tolist():
                return False
            if checkers.check_invariants(cfg, r):
                return False
        for seed in range(8):
            # marked scalars (some written on the device) and device-valid entry copies
            cfg = synth.mark_scalars(synth.random_dag(100 + seed, 9, 65, p_loop_entry=0.3 if seed % 2 else 0.0),
                                     seed, frac=0.5, read_only_frac=0.6)
            m = synth.var_mask(cfg.n_vars)
            rng = np.random.Generator(np.random.PCG64(seed))
            evd = np.array([int(x) for x in rng.integers(0, 1 << 62, size=cfg.wd)], dtype=np.uint64) & m
            cfg.entry_valid_d = evd
            cfg.entry_valid_h = m.copy()
            cfg.exit_live_d = np.array([int(x) for x in rng.integers(0, 1 << 62, size=cfg.wd)], dtype=np.uint64) & m
            r = oracle.solve(cfg)
            nu_h, nu_d = checkers.mop_nu(cfg)
            if checkers.rows_int(r["nu_h"]) != nu_h or checkers.rows_int(r["nu_d"]) != nu_d:
                return False
            if (checkers.rows_int(r["ave_h"]), checkers.rows_int(r["ave_d"])) != \
                    checkers.mop_valid(cfg, [nu_h, nu_d], [{}, {}]):
                return False
            if checkers.check_invariants(cfg, r):
                return False
        for seed in range(3):
            for cfg in (synth.c1(seed), synth.mark_scalars(synth.c1(seed), 7 + seed)):
                r = oracle.solve(cfg)
                if checkers.check_invariants(cfg, r):
                    return False
                errs, _ = checkers.simulate_paths(cfg, r, walks=30, seed=seed)
                if errs:
                    return False
    except oracle.OracleError:
        return False
    return True


def test_unmutated_passes():
    assert run_pins()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert old in src, "mutation site not found: " + name
    mut = tmp_path / ("oracle_%s.c" % name)
    mut.write_text(src.replace(old, new, 1))
    so = tmp_path / ("liboracle_%s.so" % name)
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-o", str(so), str(mut)])
    prev = oracle.use_library(str(so))
    try:
        assert not run_pins(), "the pins did not catch mutant " + name
    finally:
        oracle.restore_library(prev)
