"""CPU reference (test infrastructure only): per-Gaussian projection in float64.

Only tests, the smoke check and the CPU-baseline timing use this package; the
product path never imports it.

Follows the 3DGS preliminaries of the paper (Appendix A, Eq. `gaussian`): a
Gaussian with centre mu, covariance Sigma = R S S^T R^T built from a rotation
quaternion and per-axis scales, an opacity and a view-dependent SH colour is
projected to a screen-space ellipse.  The paper keeps the standard 3DGS
parameterisation and does not restate its constants; the readings used here
(EWA screen-space Jacobian, 0.3 px^2 low-pass dilation, 3-sigma radius, 16x16
tiles, real SH of degree 3 with the Condon-Shortley phase, +0.5 colour offset
clamped at zero) are the ones every test pins.

Every quantity is a plain vectorised float64 torch expression, so that
`torch.autograd` provides the exact derivative of each step; discrete decisions
(culling, clamps, integer radius and tile rectangle) carry zero derivative.
"""
from __future__ import annotations

import math

import torch

TILE = 16
DILATION = 0.3          # px^2 added to the screen covariance diagonal
JAC_CLAMP = 1.3         # off-axis clamp, in units of the half field of view
SH_DEGREE = 3


def _double(x):
    if isinstance(x, torch.Tensor):
        return x.to(torch.float64)
    return torch.as_tensor(x, dtype=torch.float64)


# --------------------------------------------------------------------------
# Real spherical harmonics (textbook definition)
# --------------------------------------------------------------------------
def sh_basis(dirs: torch.Tensor, degree: int = SH_DEGREE) -> torch.Tensor:
    """Real orthonormal spherical harmonics Y_lm of unit directions.

    dirs: (..., 3) unit vectors (x, y, z) with z = cos(theta).
    Returns (..., (degree+1)^2) with column l*l + l + m.

    Y_lm = sqrt(2) K_lm Q_l^m(z) Re((x+iy)^m)      m > 0
         = K_l0 Q_l^0(z)                             m = 0
         = sqrt(2) K_l|m| Q_l^|m|(z) Im((x+iy)^|m|)  m < 0
    where K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and
    P_l^m(z) = (1-z^2)^(m/2) Q_l^m(z) is the associated Legendre function
    including the Condon-Shortley phase (-1)^m, so that
    sin^m(theta) e^{i m phi} = (x + i y)^m.  Q obeys the standard recurrences
    Q_m^m = (-1)^m (2m-1)!!,  Q_{m+1}^m = (2m+1) z Q_m^m,
    (l-m) Q_l^m = (2l-1) z Q_{l-1}^m - (l+m-1) Q_{l-2}^m.
    """
    x, y, z = dirs[..., 0], dirs[..., 1], dirs[..., 2]
    L = degree
    # Q[l][m]
    Q = [[None] * (L + 1) for _ in range(L + 1)]
    for m in range(L + 1):
        dfact = 1.0
        for k in range(1, 2 * m, 2):
            dfact *= k
        Q[m][m] = torch.full_like(z, ((-1.0) ** m) * dfact)
        if m + 1 <= L:
            Q[m + 1][m] = (2 * m + 1) * z * Q[m][m]
        for l in range(m + 2, L + 1):
            Q[l][m] = ((2 * l - 1) * z * Q[l - 1][m] - (l + m - 1) * Q[l - 2][m]) / (l - m)
    # (x + i y)^m
    re = [torch.ones_like(x)]
    im = [torch.zeros_like(x)]
    for m in range(1, L + 1):
        re.append(re[-1] * x - im[-1] * y)
        im.append(re[-2] * y + im[-1] * x)
    cols = []
    for l in range(L + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            if m == 0:
                cols.append(K * Q[l][0])
            elif m > 0:
                cols.append(math.sqrt(2.0) * K * Q[l][am] * re[am])
            else:
                cols.append(math.sqrt(2.0) * K * Q[l][am] * im[am])
    return torch.stack(cols, dim=-1)


def quat_to_rotmat(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of a unit quaternion q = (w, x, y, z), shape (N, 3, 3)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = torch.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y),
    ], dim=-1)
    return R.reshape(-1, 3, 3)


def floordiv(a: torch.Tensor, b: int) -> torch.Tensor:
    return torch.div(a, b, rounding_mode="floor")


def tile_rect(mean2d: torch.Tensor, radius: torch.Tensor, width: int, height: int):
    """Integer tile rectangle [tx0, tx1) x [ty0, ty1) covering every pixel whose
    sample point lies within `radius` of the mean along x and along y."""
    TX = (width + TILE - 1) // TILE
    TY = (height + TILE - 1) // TILE
    xi = torch.floor(mean2d[:, 0]).to(torch.int64)
    yi = torch.floor(mean2d[:, 1]).to(torch.int64)
    r = radius.to(torch.int64)
    tx0 = torch.clamp(floordiv(xi - r, TILE), 0, TX)
    tx1 = torch.clamp(floordiv(xi + r, TILE) + 1, 0, TX)
    ty0 = torch.clamp(floordiv(yi - r, TILE), 0, TY)
    ty1 = torch.clamp(floordiv(yi + r, TILE) + 1, 0, TY)
    return tx0, tx1, ty0, ty1


def project(params: dict, cam, requires_grad: bool = False):
    """Project every Gaussian of `params` into camera `cam`.

    params: mean [3][N], log_scale [3][N], quat [4][N], opacity_logit [N],
            sh [16][3][N] (numpy or torch; converted to float64 leaves).
    cam:    object with width, height, fx, fy, cx, cy, R (3x3), t (3,), znear.

    Returns (leaves, out).  `leaves` are the float64 parameter tensors (with
    requires_grad when asked); `out` holds per-Gaussian float64 tensors
    mean2d (N,2), depth (N,), conic (N,3) = (a', b', c') of the inverse screen
    covariance, opacity (N,), rgb (N,3), and the integer radius (N,),
    tiles_touched (N,), the tile rectangle and rgb clamp bits (N,3).
    Culled Gaussians have radius 0 and tiles_touched 0.
    """
    leaves = {k: _double(params[k]).clone().detach().requires_grad_(requires_grad)
              for k in ("mean", "log_scale", "quat", "opacity_logit", "sh")}
    mean = leaves["mean"].T                      # (N,3)
    scale = torch.exp(leaves["log_scale"].T)     # (N,3)
    q = leaves["quat"].T
    qn = q / torch.linalg.norm(q, dim=1, keepdim=True)
    opacity = torch.sigmoid(leaves["opacity_logit"])
    sh = leaves["sh"].permute(2, 0, 1)           # (N,16,3)

    Rw = _double(cam.R).reshape(3, 3)
    tw = _double(cam.t).reshape(3)
    # Covariance Sigma = R S S^T R^T = M M^T with M = R S
    Rq = quat_to_rotmat(qn)
    M = Rq * scale[:, None, :]
    Sigma = M @ M.transpose(1, 2)
    # Camera-space centre
    tc = mean @ Rw.T + tw
    tx, ty, tz = tc[:, 0], tc[:, 1], tc[:, 2]
    in_front = tz > cam.znear
    tz_safe = torch.where(in_front, tz, torch.ones_like(tz))
    # EWA Jacobian of the perspective map at the centre, off-axis clamped
    limx = JAC_CLAMP * (cam.width / 2.0) / cam.fx
    limy = JAC_CLAMP * (cam.height / 2.0) / cam.fy
    txc = torch.clamp(tx / tz_safe, -limx, limx) * tz_safe
    tyc = torch.clamp(ty / tz_safe, -limy, limy) * tz_safe
    zero = torch.zeros_like(tz)
    J = torch.stack([
        cam.fx / tz_safe, zero, -cam.fx * txc / (tz_safe * tz_safe),
        zero, cam.fy / tz_safe, -cam.fy * tyc / (tz_safe * tz_safe),
    ], dim=-1).reshape(-1, 2, 3)
    T = J @ Rw                                    # (N,2,3)
    S2 = T @ Sigma @ T.transpose(1, 2)
    a = S2[:, 0, 0] + DILATION
    b = S2[:, 0, 1]
    c = S2[:, 1, 1] + DILATION
    det = a * c - b * b
    ok = in_front & (det > 0)
    det_safe = torch.where(ok, det, torch.ones_like(det))
    conic = torch.stack([c / det_safe, -b / det_safe, a / det_safe], dim=-1)
    mean2d = torch.stack([cam.fx * tx / tz_safe + cam.cx, cam.fy * ty / tz_safe + cam.cy], dim=-1)
    # 3-sigma radius of the larger eigenvalue
    with torch.no_grad():
        mid = 0.5 * (a + c)
        lam = mid + torch.sqrt(torch.clamp(mid * mid - det, min=0.0))
        radius = torch.ceil(3.0 * torch.sqrt(torch.clamp(lam, min=0.0))).to(torch.int64)
        radius = torch.where(ok, radius, torch.zeros_like(radius))
        tx0, tx1, ty0, ty1 = tile_rect(mean2d.detach(), radius, cam.width, cam.height)
        touched = (tx1 - tx0) * (ty1 - ty0)
        vis = ok & (touched > 0)
        radius = torch.where(vis, radius, torch.zeros_like(radius))
        touched = torch.where(vis, touched, torch.zeros_like(touched))
    # View-dependent colour
    campos = -(Rw.T @ tw)
    d = mean - campos
    d = d / torch.linalg.norm(d, dim=1, keepdim=True)
    Y = sh_basis(d)                               # (N,16)
    rgb_raw = (Y[:, :, None] * sh).sum(dim=1) + 0.5
    clamp_bits = (rgb_raw < 0).detach()
    rgb = torch.clamp(rgb_raw, min=0.0)
    out = dict(mean2d=mean2d, depth=tz, conic=conic, opacity=opacity, rgb=rgb,
               radius=radius, tiles_touched=touched, visible=vis,
               rect=torch.stack([tx0, tx1, ty0, ty1], dim=-1), clamp_bits=clamp_bits,
               lam=lam.detach(), det=det.detach())
    return leaves, out
