"""Copy of a known number of bytes, used to calibrate memory counters.

`python calib.py [MiB]` copies a device buffer of the
given size (default 512 MiB) once after a warm-up copy, so a hardware-counter
run over it (FETCH_SIZE / WRITE_SIZE per dispatch) can be compared with the
known byte count and the ratio applied to other kernels' counter readings.
"""
import sys


def main(mib: int = 512):
    import torch
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    src.fill_(1)
    dst.copy_(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {n} bytes", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 512)
