"""Counter calibration: runs the library's plain copy kernel on a buffer of known
size, so that a hardware-counter profile of this script (FETCH_SIZE, WRITE_SIZE)
gives the ratio between those counters and the bytes actually moved.

    python -m paper_2511_09413_amd.calibrate [--mib 256] [--reps 4]

Each repetition copies --mib MiB (read --mib MiB, write --mib MiB).
"""
import argparse
import ctypes as C
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=256)
    ap.add_argument("--reps", type=int, default=4)
    args = ap.parse_args()
    import torch
    import paper_2511_09413_amd as kmc
    L = kmc.lib()
    L.kmc_calib_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
    L.kmc_calib_copy.restype = C.c_int
    n = args.mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    for _ in range(args.reps):
        kmc._check(L.kmc_calib_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), n, C.c_void_p(st)))
    torch.cuda.synchronize()
    assert bool((dst == 1).all())
    print(f"copied {args.reps} x {args.mib} MiB", flush=True)


if __name__ == "__main__":
    main()
