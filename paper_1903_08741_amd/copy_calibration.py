"""Plain device-to-device copy of known size, the calibration kernel for HBM counters.

Run under ``rocprofv3 --pmc FETCH_SIZE`` (and separately ``WRITE_SIZE``): three copies
of a 1 GiB float32 tensor, so each copy dispatch reads and writes exactly 1 GiB.  The
ratio of the counter reading to 1048576 KB is the scale applied to the solver kernels.
"""
import torch


def main():
    a = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied 3 x 1 GiB", flush=True)


if __name__ == "__main__":
    main()
