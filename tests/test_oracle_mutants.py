"""The pins catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of oracle.c (on the CPU, in a temporary
directory), builds it, routes the oracle binding through it and runs the pin
suite: at least one pin must fail.  The real oracle is untouched.
"""
import inspect
import multiprocessing
import os


import oracle
import test_oracle_pins as pins

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()

# (name, text in oracle.c, replacement)
MUTANTS = [
    ("eq1 without +0.5",
     "* (g->feed_spacing_m / g->c0) * g->sin_theta_ns[m] + 0.5;",
     "* (g->feed_spacing_m / g->c0) * g->sin_theta_ns[m];"),
    ("eq1 truncation instead of floor",
     "int64_t k = (int64_t)floor(t);", "int64_t k = (int64_t)t;"),
    ("nibbles swapped",
     "out[2 * i] = (double)((int)(in[i] >> 4) - 8);\n        out[2 * i + 1] = (double)((int)(in[i] & 15) - 8);",
     "out[2 * i] = (double)((int)(in[i] & 15) - 8);\n        out[2 * i + 1] = (double)((int)(in[i] >> 4) - 8);"),
    ("decode offset 7",
     "out[2 * i] = (double)((int)(in[i] >> 4) - 8);", "out[2 * i] = (double)((int)(in[i] >> 4) - 7);"),
    ("N-S conjugate phase",
     "re += xr * wr - xi * wi;\n            im += xr * wi + xi * wr;\n            r += km;",
     "re += xr * wr + xi * wi;\n            im += -xr * wi + xi * wr;\n            r += km;"),
    ("N-S phase step off by one feed",
     "            r += km;\n            if (r >= n_bins) r -= n_bins;",
     "            r += km + (n == 0 ? km : 0);\n            while (r >= n_bins) r -= n_bins;"),
    ("E-W weight sign",
     "w[2 * (j * g->n_cyl + c) + 1] = -sin(a);", "w[2 * (j * g->n_cyl + c) + 1] = sin(a);"),
    ("E-W weights transposed",
     "double wr = w[2 * (j * n_cyl + c)], wi = w[2 * (j * n_cyl + c) + 1];",
     "double wr = w[2 * (c * n_ew + j)], wi = w[2 * (c * n_ew + j) + 1];"),
    ("no centre shift of sub-channels",
     "int32_t q = (s + L / 2) % L;", "int32_t q = s;"),
    ("time DFT sign",
     "re += b[2 * t] * wr - b[2 * t + 1] * wi;\n            im += b[2 * t] * wi + b[2 * t + 1] * wr;",
     "re += b[2 * t] * wr + b[2 * t + 1] * wi;\n            im += -b[2 * t] * wi + b[2 * t + 1] * wr;"),
    ("power drops imaginary part",
     "u[2 * s] * u[2 * s] + u[2 * s + 1] * u[2 * s + 1];", "u[2 * s] * u[2 * s];"),
    ("last block not integrated",
     "                for (int32_t blk = 0; blk < T / L; ++blk) {\n                    size_t ob = (((size_t)p * NJ + j) * NM + m) * T + (size_t)blk * L;\n                    orc_upchan_tab(L, roots_l, &B[2 * ob], u);\n                    for (int32_t s = 0; s < L; ++s) {\n                        int32_t q",
     "                for (int32_t blk = 0; blk < T / L - 1; ++blk) {\n                    size_t ob = (((size_t)p * NJ + j) * NM + m) * T + (size_t)blk * L;\n                    orc_upchan_tab(L, roots_l, &B[2 * ob], u);\n                    for (int32_t s = 0; s < L; ++s) {\n                        int32_t q"),
    ("complex beams written conjugated",
     "                        out[2 * o + 1] = u[2 * s + 1];", "                        out[2 * o + 1] = -u[2 * s + 1];"),
    ("one polarisation only",
     "            for (int32_t p = 0; p < NP; ++p)\n                for (int32_t blk",
     "            for (int32_t p = 0; p < 1; ++p)\n                for (int32_t blk"),
    ("input index feed-major",
     "int64_t i = ((int64_t)c * NF + n) * NP + p;", "int64_t i = ((int64_t)c * NP + p) * NF + n;"),
    ("8-bit code truncated instead of rounded",
     "float x = rintf(fmaf((float)P[i], scale[i], offset[i]));",
     "float x = truncf(fmaf((float)P[i], scale[i], offset[i]));"),
    ("8-bit code saturating at 254",
     "if (x > 255.0f) x = 255.0f;", "if (x > 254.0f) x = 254.0f;"),
    ("fine bins grouped without centring",
     "int32_t q = ((qf + G / 2) / G) % nq;", "int32_t q = (qf / G) % nq;"),
    ("fine bins grouped one fine channel high",
     "int32_t q = ((qf + G / 2) / G) % nq;", "int32_t q = ((qf + G / 2 - 1) / G) % nq;"),
    ("beam index N-S major",
     "out[((size_t)j * NM + m) * L + q] +=", "out[((size_t)m * NJ + j) * L + q] +="),
]

# Mistakes that a pin stated from the paper (not a restatement of the oracle's own
# rule) must catch: mutant name -> that pin.
REQUIRED_CATCHER = {
    "fine bins grouped without centring": "test_upchan128_tone_grouping",
    "fine bins grouped one fine channel high": "test_upchan128_tone_grouping",
}

PIN_TESTS = [(name, fn) for name, fn in inspect.getmembers(pins, inspect.isfunction)
             if name.startswith("test_")]


def _run_pins(oracle_mod):
    failed = []
    for name, fn in PIN_TESTS:
        kwargs = {"oracle_mod": oracle_mod} if "oracle_mod" in inspect.signature(fn).parameters else {}
        try:
            fn(**kwargs)
        except Exception:
            failed.append(name)
    return failed


def _mutant_worker(job):
    """Build one mutant in its own directory and run every pin against it."""
    name, old, new, workdir = job
    lib = oracle.build_variant(SRC.replace(old, new), os.path.join(workdir, "liboracle_mutant.so"))
    with oracle.use_library(lib):
        return name, _run_pins(oracle)


def test_pins_catch_planted_mistakes(tmp_path):
    for name, old, _ in MUTANTS:
        assert SRC.count(old) == 1, "mutation anchor not unique: %s" % name
    jobs = []
    for i, (name, old, new) in enumerate(MUTANTS):
        d = tmp_path / ("m%02d" % i)
        d.mkdir()
        jobs.append((name, old, new, str(d)))
    workers = max(1, min(8, (os.cpu_count() or 2) // 2))
    ctx = multiprocessing.get_context("spawn")
    with ctx.Pool(workers) as pool:
        results = pool.map(_mutant_worker, jobs)
    missed = []
    for name, failed in results:
        print("%s: caught by %s" % (name, failed))
        if not failed:
            missed.append(name)
        if name in REQUIRED_CATCHER and REQUIRED_CATCHER[name] not in failed:
            missed.append("%s (not by %s)" % (name, REQUIRED_CATCHER[name]))
    assert not missed, "no pin detects: %s" % missed


def test_unmodified_oracle_passes_all_pins():
    assert _run_pins(oracle) == []
