"""Plain device copy of a known size, for calibrating rocprofv3 traffic
counters (FETCH_SIZE / WRITE_SIZE in KiB per dispatch): the copy moves
exactly 256 MiB in and 256 MiB out.  Not collected by pytest.

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -- python3 tests/prof_copy_calibration.py
"""

import torch

N = 256 * 1024 * 1024 // 4
x = torch.ones(N, dtype=torch.float32, device="cuda")
y = torch.empty_like(x)
for _ in range(3):
    y.copy_(x)
torch.cuda.synchronize()
print("copied", 4 * N, "bytes x 3")
