"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer: the
oracle, the compiler's host lowering and the bounds-checked CPU replay of
the lowered tables are built with -fsanitize=address,undefined (g++/gcc only,
no device code) and run on a set of circuits (every gate kind, surface and
bivariate bicycle codes, a concatenated branch, degenerate and malformed
texts). Any sanitizer report aborts the run; the driver program also checks
the replayed signatures against the oracle's (see sanitize_main.cpp)."""

import os
import shutil
import subprocess

import pytest

from workloads import (bit_flip_code_fig1, bivariate_bicycle_memory, iceberg_surface_batch, log_uniform_rates,
                       mirror_circuit, repetition_code_memory, rotated_surface_code_memory)

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2604_16613_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc and g++")


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    obj = str(d / "oracle.o")
    exe = str(d / "sanitize_main")
    subprocess.run(["gcc", "-std=c11", "-pthread", *SAN, "-c", os.path.join(ROOT, "oracle", "gp_oracle.c"),
                    "-o", obj], check=True)
    subprocess.run(["g++", "-std=c++17", "-pthread", *SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    os.path.join(HERE, "sanitize_main.cpp"), os.path.join(HERE, "host_check.cpp"),
                    os.path.join(CSRC, "lower.cpp"), obj, "-o", exe, "-lm"], check=True)
    return d, exe


def test_host_code_is_clean_under_sanitizers(sanitized):
    d, exe = sanitized
    circuits = {
        "fig1": bit_flip_code_fig1().text,
        "rep7": repetition_code_memory(7, 5, p_data=0.01, p_meas=0.02, p2=0.03, p1=0.04,
                                       data_noise="DEPOLARIZE1").text,
        "sc3": rotated_surface_code_memory(3, 3).text,
        "sc5": rotated_surface_code_memory(5, 5).text,
        "sc9": rotated_surface_code_memory(9, 9).text,
        "bb144": bivariate_bicycle_memory().text,
        "iceberg3": iceberg_surface_batch(3, n_branches=1, seed=5)[0].text,
        "empty": "",
        "noise_free": "R 0 1\nCX 0 1\nM 0 1\nDETECTOR rec[-1] rec[-2]\n",
        "no_detectors": "R 0\nX_ERROR(0.1) 0\nM 0\n",
        "only_silent": "R 0\nZ_ERROR(0.1) 0\nM 0\nDETECTOR rec[-1]\n",
    }
    for s in range(4):
        circuits[f"mirror{s}"] = mirror_circuit(5, 6, s, x_basis=[s % 5, (s + 1) % 5]).text
    bad = {
        "odd_cx": "CX 0\n",
        "repeat": "REPEAT 3 {\nH 0\n}\n",
        "bad_rate": "X_ERROR(0.7) 0\n",
        "bad_record": "M 0\nDETECTOR rec[-2]\n",
        "unknown": "FOO 1 2\n",
        "bad_arg": "DEPOLARIZE1(abc) 0\n",
    }
    files = []
    for name, text in circuits.items():
        p = d / f"{name}.stim"
        p.write_text(text)
        files.append(str(p))
    for name, text in bad.items():
        p = d / f"{name}.bad"
        p.write_text(text)
        files.append(str(p))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, *files], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert "batch of" in r.stdout


def test_lowering_threads_are_race_free_under_tsan(tmp_path):
    """The host lowering built with -fsanitize=thread: large texts (the
    tokenizer threads claiming chunks while the scheduling thread works
    through them, the channel-table and injection-list threads), a multi-chunk
    text below the thread size, and large texts with an error early, in the
    middle or at the end (tokenizer errors and schedule errors: the scheduling
    thread stops while tokenizer threads still run). Any data race fails the
    run."""
    exe = str(tmp_path / "tsan_lower")
    subprocess.run(["g++", "-std=c++17", "-pthread", "-fsanitize=thread", "-g", "-O1", "-I",
                    os.path.join(ROOT, "include"), "-I", CSRC, os.path.join(HERE, "tsan_lower_main.cpp"),
                    os.path.join(CSRC, "lower.cpp"), "-o", exe], check=True)
    big = rotated_surface_code_memory(17, 17).text
    lines = big.split("\n")
    n = len(lines)
    files = {
        "sc17.stim": big,
        "sc13.stim": rotated_surface_code_memory(13, 13).text,
        "bb144.stim": bivariate_bicycle_memory().text,
        "early.bad": "\n".join(lines[:50] + ["FOO 1"] + lines[50:]),
        "middle.bad": "\n".join(lines[:n // 2] + ["CX 0"] + lines[n // 2:]),
        "late.bad": "\n".join(lines[:n - 20] + ["H rec[-1]"] + lines[n - 20:]),
    }
    paths = []
    for name, text in files.items():
        p = tmp_path / name
        p.write_text(text)
        paths.append(str(p))
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:exitcode=66")
    r = subprocess.run([exe, *paths], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert "WARNING: ThreadSanitizer" not in r.stderr
    assert r.stdout.count("lowered ") == 3 and r.stdout.count("rejected ") == 3
