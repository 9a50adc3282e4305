"""Host-side checks of the C ABI that need no GPU: the library loads, exports every function that
include/nbody.h declares, and rejects invalid systems before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1003_3896_amd import inputs, nbody

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "nbody.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nbody_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_abi():
    names = declared_functions()
    for required in ("nbody_accel", "nbody_step_leapfrog", "nbody_step_sym6", "nbody_energy", "nbody_create",
                     "nbody_destroy", "nbody_workspace_bytes", "nbody_substep", "nbody_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = nbody.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) <= set(nbody.EXPORTS) | {"nbody_set_tile", "nbody_get_tile"}


def test_workspace_bytes_and_interactions():
    b = inputs.c4(B=6, lo=256, hi=4096)
    s = nbody.system_from_batch(b)
    ws = nbody.nbody_workspace_bytes(None, s)
    assert ws >= 8 * b.n and ws % 256 == 0
    assert nbody.nbody_interactions(s) == b.interactions_per_eval()
    # workspace does not depend on precision, except for the local mode's sort buffers
    for p in ("fp32", "fp32c", "fp64"):
        assert nbody.nbody_workspace_bytes(None, s.with_prec(p)) == ws
    wdl = nbody.nbody_workspace_bytes(None, s.with_prec("fp32dl"))
    assert wdl >= ws + 48 * b.n and wdl <= nbody.nbody_workspace_bytes_max(b.n, b.B)
    # the batch-independent bound covers it, and covers adversarial batches of the same totals
    bound = nbody.nbody_workspace_bytes_max(b.n, b.B)
    assert bound >= ws
    for sizes in ([1] * (b.B - 1) + [b.n - b.B + 1], [b.n // b.B] * (b.B - 1) + [b.n - (b.n // b.B) * (b.B - 1)],
                  [4096] * (b.n // 4096)):
        offs = np.concatenate([[0], np.cumsum(sizes)])
        sys2 = nbody.System(offs, 1e-3)
        assert nbody.nbody_workspace_bytes(None, sys2) <= nbody.nbody_workspace_bytes_max(offs[-1], len(sizes))


@pytest.mark.parametrize("bad", [
    dict(offsets=[0, 10, 5], eps=[0.1, 0.1]),            # decreasing
    dict(offsets=[0, 10, 10], eps=[0.1, 0.1]),           # empty cluster
    dict(offsets=[1, 10], eps=[0.1]),                    # offsets[0] != 0
    dict(offsets=[0, 10], eps=[-1.0]),                   # negative eps
    dict(offsets=[0, 10], eps=[float("nan")]),           # nan eps
    dict(offsets=[0, 10], eps=[0.1], G=0.0),             # G <= 0
    dict(offsets=[0, 10], eps=[0.1], G=float("inf")),    # G inf
    dict(offsets=[0, 10], eps=[0.1], prec=7),            # unknown mode
    dict(offsets=[0, 10], eps=[0.1], field=[1], galaxy=(1, 0.7, 4.5, 3.0, 0.0, 0.7, 12.0)),  # bd = 0
    dict(offsets=[0, 10], eps=[0.1], field=[1], galaxy=(1, 0.7, 4.5, 3.0, 0.28, 0.7, float("nan"))),
    dict(offsets=[0, 10], eps=[0.1], field=[1], galaxy=(1, 0.7, 4.5, 3.0, 0.28, 0.7, 12.0, -1.0, 0.0)),  # Mbh < 0
    dict(offsets=[0, 10], eps=[0.1], field=[1], galaxy=(1, 0.7, 4.5, 3.0, 0.28, 0.7, 12.0, 5.0, float("inf"))),
    dict(offsets=[0, 10], eps=[0.1], field=[1], galaxy=(1, 0.7, 4.5, 3.0, 0.28, 0.7, 12.0, 0, 0, 2, 0, 0, 0)),  # model
    dict(offsets=[0, 10], eps=[0.1], field=[1], galaxy=(606, 0.39, 3690, 5.3, 0.25, 0, 0, 0, 0, 1, 4615, 0.0, 100)),
    dict(offsets=[0, 10], eps=[0.1], field=[1], galaxy=(606, 0.39, 3690, 5.3, 0.25, 0, 0, 0, 0, 1, 4615, 12, 0.0)),
    dict(offsets=[0, 10], eps=[0.1], field=[1], galaxy=(606, 0.39, 3690, 5.3, 0.25, 0, 0, 0, 0, 1, -1.0, 12, 100)),
])
def test_invalid_systems_rejected_on_host(bad):
    s = nbody.System(**bad)
    with pytest.raises(nbody.NBodyError) as ei:
        nbody.nbody_workspace_bytes(None, s)
    assert ei.value.code == nbody.NB_ERR_ARG
    assert nbody.nbody_interactions(s) == -1


def test_null_context_rejected():
    s = nbody.System([0, 4], [0.1])
    for fn, args in ((nbody.nbody_accel, (None, s, 8, 8, 8, None, 256, 1 << 20, 0)),
                     (nbody.nbody_step_leapfrog, (None, s, 8, 8, 8, 8, 0.1, 1, 256, 1 << 20, 0)),
                     (nbody.nbody_step_sym6, (None, s, 8, 8, 8, 8, 0.1, 1, 256, 1 << 20, 0)),
                     (nbody.nbody_energy, (None, s, 8, 8, 8, 8, 256, 1 << 20, 0))):
        with pytest.raises(nbody.NBodyError) as ei:
            fn(*args)
        assert ei.value.code == nbody.NB_ERR_ARG
        assert "context" in str(ei.value)
    with pytest.raises(nbody.NBodyError):
        nbody.nbody_create(-1)


def test_oracle_and_library_share_nothing():
    """The HIP library and the oracle are independent builds: neither links or names the other."""
    import oracle
    src_dir = os.path.join(ROOT, "paper_1003_3896_amd")
    for dirpath, _, files in os.walk(src_dir):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "nbody_oracle" not in txt and "liboracle" not in txt, f
    osrc = open(os.path.join(ROOT, "oracle", "nbody_oracle.c")).read()
    assert "nb_internal" not in osrc and "nbody.h" not in osrc


def test_workspace_bound_holds_for_random_batches():
    rng = np.random.default_rng(11)
    for _ in range(300):
        B = int(rng.integers(1, 40))
        sizes = np.exp(rng.uniform(0, np.log(70000), B)).astype(np.int64) + 1
        offs = np.concatenate([[0], np.cumsum(sizes)])
        prec = ("fp32ds", "fp32dl", "fp64")[int(rng.integers(0, 3))]
        ws = nbody.nbody_workspace_bytes(None, nbody.System(offs, 1e-3, prec=prec))
        cap = int(offs[-1]) + int(rng.integers(0, 1000))
        assert ws <= nbody.nbody_workspace_bytes_max(cap, B + int(rng.integers(0, 5)))


def test_workspace_bound_at_split_boundaries():
    """Single clusters and batches at the sizes where the number of j-ranges changes (2^15, 2^21)
    stay within the batch-independent bound in every precision mode."""
    for sizes in ([32767], [32768], [262144], [2 ** 21], [2 ** 21 + 1], [3_000_000], [32768] * 40,
                  [255, 256, 32767, 32768, 65536]):
        offs = np.concatenate([[0], np.cumsum(sizes)])
        for prec in ("fp32ds", "fp32dl", "fp64"):
            ws = nbody.nbody_workspace_bytes(None, nbody.System(offs, 1e-3, prec=prec))
            assert ws <= nbody.nbody_workspace_bytes_max(int(offs[-1]), len(sizes)), (sizes, prec)


def test_second_galaxy_model_accepted_and_deferred_clusters_fit_the_bound():
    """The Allen & Santillan model needs no vh or dh; its field clusters are finished by the combine
    pass, so even unsplit ones take partial-sum rows, which the batch-independent bound covers."""
    from paper_1003_3896_amd import inputs
    offs = np.array([0, 1, 3, 203, 458, 714, 1714, 5714])
    for fld in ([1] * 7, [1, 0, 1, 0, 1, 0, 1]):
        s = nbody.System(offs, 1e-3, fld, 1.0, inputs.ALLEN_SANTILLAN)
        ws = nbody.nbody_workspace_bytes(None, s)
        s0 = nbody.System(offs, 1e-3, fld, 1.0, inputs.GALAXY)
        assert ws > nbody.nbody_workspace_bytes(None, s0)   # the deferred clusters' partial rows
        assert ws <= nbody.nbody_workspace_bytes_max(int(offs[-1]), len(offs) - 1)
    big = nbody.System([0, 5_000_000], 1e-3, [1], 1.0, inputs.ALLEN_SANTILLAN)
    assert nbody.nbody_workspace_bytes(None, big) <= nbody.nbody_workspace_bytes_max(5_000_000, 1)


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes structures of the binding have the sizes and field offsets that a C compiler gives
    the header's structures (a layout drift would pass wrong values silently)."""
    import subprocess
    structs = {"nbody_galaxy": nbody.nbody_galaxy, "nbody_system": nbody.nbody_system, "nbody_tile": nbody.nbody_tile}
    src = ['#include <stddef.h>', '#include <stdio.h>', '#include "nbody.h"', 'int main(void) {']
    for name, cls in structs.items():
        src.append('  printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for f, _ in cls._fields_:
            src.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, f, name, f))
    src += ['  return 0;', '}']
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(c)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        a, b, v = line.split()
        got[(a, b)] = int(v)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)
