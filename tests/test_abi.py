"""The C-ABI library loads and exports every entry point include/gtap.h declares."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "gtap.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gtap_[a-z_]+)\s*\(", text)))


def test_header_declares_core_calls():
    names = _declared()
    for must in ("gtap_init", "gtap_submit", "gtap_run", "gtap_result", "gtap_finalize"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2604_05982_amd import gtap
    lib = ctypes.CDLL(gtap.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(gtap.EXPORTED) == set(_declared())


def test_status_strings_without_device():
    from paper_2604_05982_amd import gtap
    assert gtap.gtap_status_string(gtap.GTAP_E_CAPACITY).startswith("frame pool")
    cfg = gtap.gtap_config_default()
    assert cfg.num_queues == 1 and cfg.deque_capacity & (cfg.deque_capacity - 1) == 0


def test_struct_layout_matches_header(tmp_path):
    """Compile the real header with gcc and compare sizes and field offsets."""
    import subprocess
    from paper_2604_05982_amd import gtap
    structs = [gtap.gtap_config, gtap.gtap_fib_args, gtap.gtap_nqueens_args, gtap.gtap_uts_args,
               gtap.gtap_kclique_args, gtap.gtap_kclique_split_args, gtap.gtap_fmm_args, gtap.gtap_fmm_result,
               gtap.gtap_cilksort_args, gtap.gtap_stats,
               gtap.gtap_error_report, gtap.gtap_trace_job, gtap.gtap_trace_result, gtap.gtap_tune_space,
               gtap.gtap_tune_report, gtap.gtap_litmus_result]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gtap.h"', "int main(void){"]
    for st in structs:
        lines.append(f'printf("{st.__name__} %zu\\n", sizeof({st.__name__}));')
        for name, _ in st._fields_:
            lines.append(f'printf("{st.__name__}.{name} %zu\\n", offsetof({st.__name__}, {name}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                   check=True).stdout.splitlines())
    for st in structs:
        assert int(got[st.__name__]) == ctypes.sizeof(st), st.__name__
        for name, _ in st._fields_:
            assert int(got[f"{st.__name__}.{name}"]) == getattr(st, name).offset, (st.__name__, name)


def test_enum_values_match_header(tmp_path):
    """Status codes, modes, kinds, DAQ policies and flags: the binding's
    constants equal the header's enumerators."""
    import subprocess
    from paper_2604_05982_amd import gtap
    text = open(os.path.join(ROOT, "include", "gtap.h")).read()
    names = sorted(set(re.findall(r"\b(GTAP_[A-Z0-9_]+)\s*=", text)))
    assert names
    lines = ['#include <stdio.h>', '#include "gtap.h"', "int main(void){"]
    lines += [f'printf("{n} %d\\n", (int){n});' for n in names]
    lines.append("return 0;}")
    src = tmp_path / "enums.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "enums"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                   check=True).stdout.splitlines())
    missing = [n for n in names if not hasattr(gtap, n)]
    assert not missing, missing
    for n in names:
        assert getattr(gtap, n) == int(got[n]), n


def test_kclique_split_buffer_size_without_device():
    """Big-frame buffer ints of a split k-clique job: a split node's state
    (a 64-bit meta word and two sets of W = ceil(D/64) 64-bit words) for
    out-degree D; 0 outside [0, 1024]."""
    from paper_2604_05982_amd import gtap
    for d in (0, 1, 40, 64, 65, 313, 1024):
        w = max((d + 63) // 64, 1)
        assert gtap.kclique_split_buffer_ints(d) == 2 + 4 * w
    assert gtap.kclique_split_buffer_ints(-1) == 0 and gtap.kclique_split_buffer_ints(1025) == 0



def test_binding_shares_torchs_hip_runtime():
    """Importing the binding before torch maps one HIP runtime, not two (the
    library resolves its libamdhip64 dependency to the copy torch loaded)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2604_05982_amd import gtap\n"
            "import torch\n"
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))") % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "1", r.stdout
