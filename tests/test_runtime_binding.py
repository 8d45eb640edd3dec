"""The library shares PyTorch's HIP runtime: loading it first (a host-only
call before any device use) must not bring a second HIP runtime into the
process, where the one that starts second finds no device."""
import os
import subprocess
import sys
import textwrap

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_one_hip_runtime_when_the_library_is_loaded_first():
    code = textwrap.dedent(f"""
        import sys
        sys.path.insert(0, {ROOT!r})
        import paper_2101_08226_amd as lib
        lib.load_library()
        names = set()
        for line in open('/proc/self/maps'):
            f = line.split()[-1]
            if 'libamdhip64' in f:
                names.add(f)
        print(len(names))
    """)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1", out.stdout
