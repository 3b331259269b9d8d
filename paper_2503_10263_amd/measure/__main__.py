"""python -m paper_2503_10263_amd.measure [peaks | copy BYTES]: build the measurement program into a
temporary directory and run it."""
import subprocess
import sys

from . import build

what = sys.argv[1] if len(sys.argv) > 1 else "peaks"
exe = build("peaks")
sys.exit(subprocess.call([exe, *sys.argv[1:]] if what == "copy" else [exe]))
