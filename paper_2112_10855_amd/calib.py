"""Calibration workload for HBM counters: a plain device-to-device copy of a
1 GiB FP32 buffer (torch's copy kernel), repeated 3 times.  Under
`rocprofv3 --pmc FETCH_SIZE` (then WRITE_SIZE) the counters of this kernel
are compared with the known 1 GiB read and 1 GiB write per dispatch to scale
the counters read for the library's kernels."""

import torch


def main():
    n = 1 << 28  # floats = 1 GiB
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("copied %d bytes x3" % (4 * n), flush=True)


if __name__ == "__main__":
    main()
