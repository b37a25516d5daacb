"""The growing colony's growth and division (Sec. 5.3) written out for the
oracle's side of the colony tests, independently of the library: lengths
are total (tip-to-tip) lengths, the shape holds the cylinder length
l = length - 2 r; a dividing cell becomes its two halves, tip to tip, each
turned about the z axis by its own angle.  Rotations come from scipy."""
import numpy as np
from scipy.spatial.transform import Rotation


def _rot(q):
    q = np.asarray(q, float)
    return Rotation.from_quat([q[1], q[2], q[3], q[0]])


def grow(shape, dl):
    out = np.array(shape, float).copy()
    out[:, 1] += dl
    return out


def divide(x, q, shape, rho, l_div, jitter):
    """Cells with l >= l_div replaced by their first half, second halves
    appended in parent order; jitter[2k], jitter[2k+1] turn the k-th
    parent's two halves.  Returns (x, q, shape, rho, number divided)."""
    x, q, shape, rho = (np.array(a, float).copy() for a in (x, q, shape, rho))
    idx = np.where(shape[:, 1] >= l_div)[0]
    nx, nq, ns, nr = [x], [q], [shape], [rho]
    for k, a in enumerate(idx):
        r, l = shape[a, 0], shape[a, 1]
        R = _rot(q[a])
        t = R.apply([1.0, 0.0, 0.0])
        h = 0.25 * (l + 2.0 * r)
        halves = []
        for d, sgn in ((0, 1.0), (1, -1.0)):
            Rd = Rotation.from_rotvec([0.0, 0.0, jitter[2 * k + d]]) * R
            v = Rd.as_quat()
            qd = np.array([v[3], v[0], v[1], v[2]])
            halves.append((x[a] + sgn * h * t, qd / np.linalg.norm(qd)))
        x[a], q[a] = halves[0]
        shape[a] = (r, 0.5 * l - r, 0.0)
        nx.append(halves[1][0][None])
        nq.append(halves[1][1][None])
        ns.append(np.array([[r, 0.5 * l - r, 0.0]]))
        nr.append(rho[a:a + 1])
    return np.concatenate(nx), np.concatenate(nq), np.concatenate(ns), np.concatenate(nr), len(idx)


def same_rotation(qa, qb):
    """Largest difference of unit quaternions up to sign, per body."""
    qa, qb = np.asarray(qa), np.asarray(qb)
    s = np.sign(np.sum(qa * qb, axis=1, keepdims=True))
    s[s == 0] = 1.0
    return np.abs(qa - s * qb).max()
