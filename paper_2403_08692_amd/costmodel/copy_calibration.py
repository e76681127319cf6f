"""Calibration kernel for the HBM byte counters: a device-to-device copy of
a known size (2 GiB read, 2 GiB written per dispatch), run under
rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) so that the counters' KiB per
dispatch can be scaled to bytes.  Usage: python -m
paper_2403_08692_amd.costmodel.copy_calibration"""
import torch

N_BYTES = 2 << 30


def main():
    a = torch.empty(N_BYTES // 8, dtype=torch.float64, device="cuda:0")
    a.fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {N_BYTES} bytes x3")


if __name__ == "__main__":
    main()
