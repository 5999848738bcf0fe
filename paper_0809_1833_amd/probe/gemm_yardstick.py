"""Yardstick for the batched correlation product: the vendor BF16 GEMM
(torch.matmul, which dispatches to hipBLASLt on ROCm) on the product's
shape, C = Psi^T R with Psi^T (M x N) and R (N x B), for the active-signal
counts a batched decode passes through.

Prints one line per B with the mean time of 200 back-to-back products and
the FLOP rate (2 M N B per product).  This is a measurement aid, not part of
the decoder: the decoder's product (k_bcorr) also keeps each signal's top 8
atoms per tile, which a plain GEMM does not.

    python -m paper_0809_1833_amd.probe.gemm_yardstick [--n 2048] [--m 8192]
"""
from __future__ import annotations

import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--m", type=int, default=8192)
    ap.add_argument("--reps", type=int, default=200)
    a = ap.parse_args()
    torch.manual_seed(0)
    psit = torch.randn(a.m, a.n, device="cuda").to(torch.bfloat16).contiguous()
    for b in (16, 32, 64, 96, 128, 192, 256):
        r = torch.randn(a.n, b, device="cuda").to(torch.bfloat16).contiguous()
        for _ in range(10):
            c = psit @ r
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.reps):
            c = psit @ r
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / a.reps * 1e3
        print(f"B {b:4d}  {us:8.2f} us  {2.0 * a.m * a.n * b / us / 1e6:7.1f} TFLOP/s", flush=True)
    del c


if __name__ == "__main__":
    main()
