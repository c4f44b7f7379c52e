"""Shared set-up of the GPU parity tests: one geometry built twice, once by the
oracle (FP64, numpy) and once by the HIP library, from the same parameters."""

from __future__ import annotations

import sys

import numpy as np
import torch

from oracle import cisor as ocisor


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make_pair(n, h, T, M, rx_radius=None, precision="c64", eps_b=1.0):
    from paper_1708_01663_amd.cisor import Cisor, plane_wave_dirs, ring
    rx_radius = n * h if rx_radius is None else rx_radius
    prob = ocisor.make_problem_2d(n, h, T, M, rx_radius, eps_b=eps_b)
    op = Cisor(n, h, plane_wave_dirs(T), ring(M, rx_radius), eps_b=eps_b, precision=precision)
    return prob, op


def to_dev(x, op, real=False):
    dt = op.rdtype if real else op.cdtype
    return torch.from_numpy(np.ascontiguousarray(x)).to(dt).to(op.device).contiguous()


def to_np(x):
    return x.detach().cpu().numpy().astype(np.complex128 if x.is_complex() else np.float64)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))
