"""Write the tile-variant cache that bench.py and users load with
Plan.autotune(path) / Batch.autotune(path): one line per (arch, grid,
precision) holding the variant of each FFT pass and the timings that chose
it, and one per (arch, precision, set of lengths) of the batched workload
holding the column and row tile variant per length.

    python -m paper_0911_1407_amd.make_tune_cache [path]

Runs on the GPU; the default path is tune_cache_<arch>.txt beside this file.
"""
import os
import sys

import torch

from . import binding, synth

GRIDS = (("sel256", None), ("big512", None), ("sel256", 128), ("plain32", None))


def main(argv):
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    path = argv[1] if len(argv) > 1 else os.path.join(os.path.dirname(__file__), f"tune_cache_{arch}.txt")
    if os.path.exists(path):
        os.remove(path)
    for name, n in GRIDS:
        inst = synth.config_instance(name, n=n)
        plan = binding.Plan(inst["n"], inst["box"], precision="mixed")
        plan.set_instance(inst)
        print(name, inst["n"], plan.autotune(path), flush=True)
        plan.close()
    # the batched workload's tile variants per grid length
    batch = binding.Batch(synth.batch_instances(count=64), precision="mixed")
    batch.autotune(path)
    batch.close()
    print(open(path).read(), end="")


if __name__ == "__main__":
    main(sys.argv)
