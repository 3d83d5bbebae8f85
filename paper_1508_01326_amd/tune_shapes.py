"""Write a launch-shape table for the current device: radic_autotune on the
given matrix shapes in both float precisions, then radic_tune_save.

    python -m paper_1508_01326_amd.tune_shapes OUT.txt M N [M N ...]

The table (device architecture, library version, and per shape and
enumeration the subsets per lane and workgroup size) is loaded with
radic_tune_load; a table of another architecture or version is refused."""
import sys

from . import binding


def main(argv):
    if len(argv) < 3 or (len(argv) - 1) % 2:
        print(__doc__, file=sys.stderr)
        return 2
    out = argv[0]
    dims = [int(x) for x in argv[1:]]
    for m, n in zip(dims[0::2], dims[1::2]):
        for prec in ("fp64", "fp32_bulk"):
            spl, block = binding.autotune(binding.RADIC_WS_DET, m, n, prec)
            print(f"{m}x{n} {prec}: subsets per lane {spl}, workgroup {block}", flush=True)
    binding.tune_save(out)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
