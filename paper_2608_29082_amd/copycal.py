"""Plain device copy of a known size, used to calibrate HBM byte counters.

    python -m paper_2608_29082_amd.copycal [MiB]

Copies a float32 buffer of the given size (default 256 MiB) five times with
torch's copy kernel; each dispatch reads and writes exactly that many bytes.
"""
import sys

import torch

mib = int(sys.argv[1]) if len(sys.argv) > 1 else 256
n = mib * (1 << 20) // 4
x = torch.randn(n, device="cuda")
y = torch.empty_like(x)
for _ in range(5):
    y.copy_(x)
torch.cuda.synchronize()
print(f"copied {mib} MiB x5")
