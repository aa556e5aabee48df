"""A plain device copy of known size, used to calibrate the HBM byte counters
(FETCH_SIZE, WRITE_SIZE) that the kernel profiles are scaled by: each dispatch of
the multiply-by-one kernel reads and writes exactly `nbytes` bytes.

    python3 -m paper_2310_13145_amd.hbm_copy [nbytes] [reps]
"""
from __future__ import annotations

import json
import sys


def main(nbytes: int = 1 << 30, reps: int = 5):
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"read_bytes_per_dispatch": 4 * n, "write_bytes_per_dispatch": 4 * n, "dispatches": reps}),
          flush=True)


if __name__ == "__main__":
    args = [int(v) for v in sys.argv[1:3]]
    main(*args)
