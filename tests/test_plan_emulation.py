"""The pass planner, checked on the host: circuits are planned as for the GPU
(register-staged passes, lane ops, SWAP relabelling, phase polynomials) and
the planned ops are replayed in planned order on a full state vector by
tests/host/plan_emulator.cpp, against the gates applied in user order."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2009_01845_amd", "csrc")


@pytest.fixture(scope="module")
def emulator(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    out = str(tmp_path_factory.mktemp("emu") / "plan_emulator")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", CSRC, "-o", out, os.path.join(HERE, "host", "plan_emulator.cpp"),
                    os.path.join(CSRC, "planner.cpp")], check=True)
    return out


@pytest.mark.parametrize("dbl", [0, 1])
@pytest.mark.parametrize("lanes", [0, 1])
@pytest.mark.parametrize("n,tile_bits,seed,mode", [
    (15, 0, s, 0) for s in range(1, 9)] + [(14, 12, s, 0) for s in range(1, 9)] + [(15, 13, 2, 0)] +
    [(n, 12, 5, 1) for n in (12, 13, 14, 15, 16)] + [(n, 12, 5, 2) for n in (12, 13, 14, 16)] +
    [(n, 0, 7, 3) for n in (12, 13, 14, 16)])
def test_planned_ops_replay_the_circuit(emulator, n, tile_bits, seed, mode, lanes, dbl):
    r = subprocess.run([emulator, str(n), str(tile_bits), str(seed), str(mode), str(lanes), str(dbl)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr


def test_lane_ops_are_planned_and_only_in_the_one_state_form(emulator):
    r = subprocess.run([emulator, "14", "12", "5", "1", "1"], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout
    one, two = r.stdout.strip().splitlines()
    assert int(one.split("lane_ops=")[1].split()[0]) > 0
    # the counter is cumulative: the two-state form adds none
    assert one.split("lane_ops=")[1].split()[0] == two.split("lane_ops=")[1].split()[0]


def test_no_lane_ops_unless_asked(emulator):
    r = subprocess.run([emulator, "14", "12", "5", "1", "0"], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout
    assert all(line.split("lane_ops=")[1].split()[0] == "0" for line in r.stdout.strip().splitlines())


@pytest.mark.parametrize("dbl,expect", [(0, 3), (1, 2)])
def test_matrix_core_blocks_on_disjoint_bits_share_passes(emulator, dbl, expect):
    # two ready blocks of the same size whose targets fit one tile run in one
    # pass: at 16 qubits the 5-qubit low/high pair and two 4-qubit pairs (only
    # the 4-qubit pairs in complex128)
    r = subprocess.run([emulator, "16", "0", "7", "3", "0", str(dbl)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout
    assert all(int(line.split("mfma_fused=")[1].split()[0]) == expect for line in r.stdout.strip().splitlines())
