"""A device copy of known size (1 GiB read, 1 GiB written) used to calibrate
rocprofv3 FETCH_SIZE / WRITE_SIZE readings: run it under the same counter
collection as the library and divide."""
import torch


def main():
    n = 1 << 28  # int32 elements: 1 GiB
    a = torch.ones(n, dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print("copied %d bytes" % (4 * n), flush=True)


if __name__ == "__main__":
    main()
