"""Point cloud to voxel grid and image-quality figures (include/sbp_image.h).

Argument marshalling only; the voxelisation and the MSE / PSNR / SSIM
reductions run in libsbp.so.
"""
from __future__ import annotations

import ctypes

import torch

from . import _abi, api
from ._abi import check, lib
from .api import _at_least, _check_balls, _exactly, _need, _p, _stream, balls_struct


def voxelize(ctx, balls, ball_off, model: api.Model, grid, B_cap=None, vox=None, stream=None):
    """sbp_voxelize: the cloud's initial pressure at the centres of `grid`'s voxels
    (a flat tensor of nx*ny*nz floats; view it as [nx, ny, nz])."""
    dev = balls["x"].device
    if vox is None:
        vox = torch.empty(grid.ncell, dtype=torch.float32, device=dev)
    cap = balls["x"].numel() if B_cap is None else int(B_cap)
    _check_balls(balls, cap)
    _exactly(_need(vox, name="vox"), grid.ncell, "vox")
    check(lib().sbp_voxelize(ctx.ptr, ctypes.byref(balls_struct(balls)),
                             _p(_need(ball_off, torch.int64, "ball_off")), cap,
                             ctypes.byref(model.struct()), ctypes.byref(grid.struct()),
                             _p(_need(vox, name="vox")), _stream(stream)))
    return vox


def metrics(ctx, img, ref, shape, scale, work=None, stream=None):
    """sbp_image_metrics: device tensor [MSE, PSNR, SSIM] (float64)."""
    nx, ny, nz = (int(s) for s in shape)
    n = nx * ny * nz
    _need(img, name="img")
    _need(ref, name="ref")
    if img.numel() != n or ref.numel() != n:
        raise ValueError("img and ref must hold nx*ny*nz values")
    if work is None:
        work = torch.empty(10 * n, dtype=torch.float32, device=img.device)
    _at_least(_need(work, name="work"), 10 * n, "work")
    out = torch.empty(3, dtype=torch.float64, device=img.device)
    check(lib().sbp_image_metrics(ctx.ptr, _p(img), _p(ref), nx, ny, nz, float(scale),
                                  _p(_need(work, name="work")), _p(out), _stream(stream)))
    return out
