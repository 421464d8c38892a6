"""Plain copy of a known size, used to calibrate the HBM byte counters of a profiler
(FETCH_SIZE and WRITE_SIZE of this kernel should read 256 MiB each)."""
import torch


def main():
    torch.cuda.set_device(0)
    x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")  # 256 MiB
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print("copy probe: 3 launches of 256 MiB read + 256 MiB written", flush=True)


if __name__ == "__main__":
    main()
