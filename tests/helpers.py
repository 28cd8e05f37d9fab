"""Small hand-built scenes for closed-form checks (no rendering arithmetic here)."""
import numpy as np

import synth


def camera(width=32, height=32, eye=(0.0, 0.0, 3.0), target=(0.0, 0.0, 0.0), fov=50.0):
    return synth.look_at_camera(eye, target, width, height, fov)


def cam_axes(cam):
    """World-space camera axes (right, down, forward) and the camera centre."""
    w2c = np.asarray(cam["w2c"], np.float64)
    R, t = w2c[:, :3], w2c[:, 3]
    return R[0], R[1], R[2], -R.T @ t


def quat_of_frame(tu, tv, n):
    return synth._quat_from_frames(np.asarray([tu], float), np.asarray([tv], float),
                                   np.asarray([n], float))[0]


def quat_rotate(q, v):
    """Rotate v by the unit quaternion q=(w,x,y,z) through Hamilton products q v q*."""
    w, x, y, z = q / np.linalg.norm(q)

    def mul(a, b):
        a0, a1, a2, a3 = a
        b0, b1, b2, b3 = b
        return np.array([a0 * b0 - a1 * b1 - a2 * b2 - a3 * b3,
                         a0 * b1 + a1 * b0 + a2 * b3 - a3 * b2,
                         a0 * b2 - a1 * b3 + a2 * b0 + a3 * b1,
                         a0 * b3 + a1 * b2 - a2 * b1 + a3 * b0])
    r = mul(mul(np.array([w, x, y, z]), np.array([0.0, *v])), np.array([w, -x, -y, -z]))
    return r[1:]


def scene_from(splats, T=2, env=None, env_levels=1, textures=None):
    """splats: list of dicts with mean, quat, scale (2), opac. textures [N,T,T,8] or None."""
    n = len(splats)
    sc = {
        "means": np.array([s["mean"] for s in splats], np.float32).reshape(n, 3),
        "quats": np.array([s["quat"] for s in splats], np.float32).reshape(n, 4),
        "scales": np.array([s["scale"] for s in splats], np.float32).reshape(n, 2),
        "opac": np.array([s["opac"] for s in splats], np.float32).reshape(n),
        "chart_of": np.arange(n, dtype=np.int32),
        "env_levels": env_levels,
    }
    if textures is None:
        textures = np.zeros((n, T, T, 8), np.float32)
        textures[..., 6] = 1.0
    sc["textures"] = np.ascontiguousarray(textures, np.float32)
    sc["tex_res"] = sc["textures"].shape[1]
    if env is None:
        env = np.ones((6, 4, 4, 3), np.float32)
    sc["env"] = np.ascontiguousarray(env, np.float32)
    return sc


def face_on_splat(cam, x, y, z0, scale=(0.1, 0.1), opac=0.8):
    """A splat in the plane z_cam = z0 whose centre is on the ray of pixel centre (x, y),
    with t_u, t_v along the camera's right and down axes."""
    right, down, fwd, o = cam_axes(cam)
    dc = np.array([(x + 0.5 - cam["cx"]) / cam["fx"], (y + 0.5 - cam["cy"]) / cam["fy"], 1.0])
    mu = o + z0 * (dc[0] * right + dc[1] * down + dc[2] * fwd)
    tu, tv = right, down
    n = np.cross(tu, tv)
    return {"mean": mu, "quat": quat_of_frame(tu, tv, n), "scale": scale, "opac": opac}
