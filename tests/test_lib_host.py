"""Host-side checks of the HIP library (no GPU needed): the shared library
loads, exports every entry point of include/tt_fde.h, and its operator
builder agrees with the oracle."""
import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from oracle import fd, fullgrid, galerkin
from paper_2403_04946_amd import tt

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "tt_fde.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void\*|void|const char\*)\s+(tt_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 25
    h = tt.lib()
    missing = [n for n in names if not hasattr(h, n)]
    assert not missing, missing
    assert set(names) == set(tt.exported_symbols())


def test_binding_constants_match_the_header():
    """Every TT_* constant of the Python binding has the value the header's
    enums give it (the binding restates them for ctypes)."""
    text = open(HEADER).read()
    header = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(TT_[A-Z0-9_]+)\s*=\s*(-?\d+)", text)}
    names = [k for k in vars(tt) if re.fullmatch(r"TT_[A-Z0-9_]+", k)]
    assert len(names) >= 20
    wrong = {k: (getattr(tt, k), header.get(k)) for k in names if header.get(k) != getattr(tt, k)}
    assert not wrong, wrong


def _zero_argument(argtype):
    if argtype in (ctypes.c_double, ctypes.c_float):
        return 0.0
    if argtype in (ctypes.c_int, ctypes.c_long, ctypes.c_longlong, ctypes.c_ulong, ctypes.c_ulonglong):
        return 0
    return None  # every pointer argument null


def test_null_handles_are_rejected_before_any_hip_call():
    """Every entry point that takes a handle returns TT_EINVAL when it and
    every other pointer argument are null and every number is zero (host
    checks only: no GPU is needed or touched)."""
    h = tt.lib()
    no_handle = {"tt_gemm_table_count", "tt_gemm_table_clear"}
    special = {"tt_last_error", "tt_ctx_stream", "tt_step_batch"}
    checked = 0
    for name in tt.exported_symbols():
        if name in no_handle or name in special:
            continue
        f = getattr(h, name)
        assert f(*[_zero_argument(a) for a in f.argtypes]) == -1, name
        checked += 1
    assert checked >= 50
    assert h.tt_last_error(None) == b"null context"
    assert h.tt_ctx_stream(None) is None
    f = h.tt_step_batch
    assert f(*[_zero_argument(a) for a in f.argtypes]) == 0  # count 0: an empty batch


# header struct -> the binding's ctypes restatement of it
STRUCTS = {
    "tt_allocator": tt.AllocatorStruct,
    "tt_op_opts": tt.OpOpts,
    "tt_cdf_opts": tt.CdfOpts,
    "tt_apply_opts": tt.ApplyOpts,
    "tt_round_report": tt.RoundReport,
    "tt_step_opts": tt.StepOpts,
    "tt_step_report": tt.StepReport,
    "tt_solve_opts": tt.SolveOpts,
    "tt_solve_report": tt.SolveReport,
}


def test_binding_structs_match_the_header(tmp_path):
    """The header compiles as plain C11, and every struct the binding passes
    through ctypes has the header's size and field offsets (printed by a
    C program built against the header with gcc)."""
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "tt_fde.h"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src, exe = tmp_path / "layout.c", tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run([gcc, "-std=c11", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        cname, field, value = line.split()
        got[(cname, field)] = int(value)
    for cname, cls in STRUCTS.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


@pytest.mark.parametrize("d", [4, 7, 20])
def test_coefficients_match_oracle(d):
    op = tt.Operator(None, d, 8, 4.0, 0.05)
    b, dm = op.coefficients()
    assert np.abs(b - galerkin.coefficient_B(d)).max() < 1e-14 * d
    assert np.abs(dm - galerkin.coefficient_D(d)).max() < 1e-14 * np.abs(dm).max()
    op.close()


def test_local_operators_match_oracle():
    n, length = 9, 3.0
    op = tt.Operator(None, 3, n, length, 0.1)
    mats = op.local_ops()
    x = fd.position(n, length)
    g = fd.first_derivative(n, length)
    l2 = fd.second_derivative(n, length)
    ref = [np.eye(n), x, g, l2, x @ g, x @ l2]
    for o in range(6):
        assert np.abs(mats[o] - ref[o]).max() < 1e-12, o
    op.close()


def mpo_dense(op, n):
    """Contract the exported automaton into the dense n^d x n^d matrix."""
    d = op.d
    mats = op.local_ops()
    R = op.ranks()
    full = np.ones((1, 1, 1), dtype=np.complex128)  # (rows, cols, bond)
    for m in range(d):
        a, b, o, c = op.site(m)
        w = np.zeros((R[m], R[m + 1], n, n), dtype=np.complex128)
        for ai, bi, oi, ci in zip(a, b, o, c):
            w[ai, bi] += ci * mats[oi]
        full = np.einsum("xya,abij->xiyjb", full, w).reshape(full.shape[0] * n, full.shape[1] * n, R[m + 1])
    return full[:, :, 0]


@pytest.mark.parametrize("d,n,nu", [(4, 5, 0.05), (5, 4, 0.0), (3, 6, 0.3)])
def test_operator_automaton_matches_oracle_operator(d, n, nu):
    length = 4.0
    op = tt.Operator(None, d, n, length, nu)
    R = op.ranks()
    assert R[0] == 1 and R[d] == 1 and max(R) <= 2 * d + 2
    dense = mpo_dense(op, n)
    prob = fullgrid.Problem(galerkin.coefficient_B(d), galerkin.coefficient_D(d), nu, n, length)
    rng = np.random.default_rng(0)
    f = rng.standard_normal((n,) * d) + 1j * rng.standard_normal((n,) * d)
    ref = prob.apply(f).ravel()
    got = dense @ f.ravel()
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    op.close()


def test_operator_ranks_at_benchmark_size():
    op = tt.Operator(None, 50, 128, 8.0, 0.01)
    R = op.ranks()
    assert R[0] == R[50] == 1 and max(R) <= 102
    op.close()


def test_invalid_arguments_are_rejected_without_a_device():
    h = tt.lib()
    out = ctypes.c_void_p()
    assert h.tt_op_create_burgers_hopf(None, 0, 8, 4.0, 0.1, ctypes.byref(out)) == -1
    assert h.tt_op_create_burgers_hopf(None, 4, 2, 4.0, 0.1, ctypes.byref(out)) == -1
    assert h.tt_op_create_burgers_hopf(None, 4, 8, -1.0, 0.1, ctypes.byref(out)) == -1
    modes = (ctypes.c_int * 4)(8, 8, 8, 8)
    assert h.tt_tensor_create(None, 4, modes, None, 0, ctypes.byref(out)) == -1
    assert h.tt_round(None, None, 0.0, None, None) == -1
    assert h.tt_ctx_create(0, None, None, None) == -1
    assert h.tt_ctx_sync(None) == -1


def test_viscous_only_operator():
    d, n, length, nu = 4, 5, 4.0, 0.2
    op = tt.Operator(None, d, n, length, nu, advection=0.0)
    assert max(op.ranks()) == 2
    dense = mpo_dense(op, n)
    prob = fullgrid.Problem(np.zeros((d, d, d)), galerkin.coefficient_D(d), nu, n, length)
    rng = np.random.default_rng(1)
    f = rng.standard_normal((n,) * d) + 1j * rng.standard_normal((n,) * d)
    ref = prob.apply(f).ravel()
    assert np.linalg.norm(dense @ f.ravel() - ref) <= 1e-12 * np.linalg.norm(ref)
    op.close()


def test_tensor_capacities_are_checked_before_the_call():
    # one capacity is spread over the interior bonds (d = 1 has none); any
    # other count is rejected on the host
    with pytest.raises(ValueError):
        tt.Tensor(None, 3, 8, [1, 4, 1])
