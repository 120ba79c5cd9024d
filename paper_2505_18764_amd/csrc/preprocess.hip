// preprocess.hip -- projection of 3D Gaussians to 2D splats and its backward, one thread per
// Gaussian (Sec. 2.1.1-2.1.2 forward; Sec. 2.1.3 "dedicated subsequent pass" backward).
// Several cameras of one scene run in one launch: the forward has grid y = view and writes each
// view's [n] outputs; the backward walks the views in order for each Gaussian and writes the sum
// of their gradients once.
#include "device.hpp"
#include "internal.hpp"

namespace gsr {

// Real spherical harmonics up to degree 3, as polynomials in the unit direction (x, y, z);
// coefficient k = l^2 + l + m. Normalisations: sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times the
// usual factors, written out.
constexpr float SH_C0 = 0.28209479177387814f;
constexpr float SH_C1 = 0.4886025119029199f;
constexpr float SH_C2A = 1.0925484305920792f;
constexpr float SH_C2B = 0.31539156525252005f;
constexpr float SH_C2C = 0.5462742152960396f;
constexpr float SH_C3A = 0.5900435899266435f;
constexpr float SH_C3B = 2.890611442640554f;
constexpr float SH_C3C = 0.4570457994644658f;
constexpr float SH_C3D = 0.3731763325901154f;
constexpr float SH_C3E = 1.445305721320277f;

__device__ __forceinline__ void sh_eval(float x, float y, float z, int deg, float Y[16]) {
    Y[0] = SH_C0;
    if (deg < 1) return;
    Y[1] = SH_C1 * y;
    Y[2] = SH_C1 * z;
    Y[3] = SH_C1 * x;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = SH_C2A * x * y;
    Y[5] = SH_C2A * y * z;
    Y[6] = SH_C2B * (2.0f * zz - xx - yy);
    Y[7] = SH_C2A * x * z;
    Y[8] = SH_C2C * (xx - yy);
    if (deg < 3) return;
    Y[9] = SH_C3A * y * (3.0f * xx - yy);
    Y[10] = SH_C3B * x * y * z;
    Y[11] = SH_C3C * y * (4.0f * zz - xx - yy);
    Y[12] = SH_C3D * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = SH_C3C * x * (4.0f * zz - xx - yy);
    Y[14] = SH_C3E * z * (xx - yy);
    Y[15] = SH_C3A * x * (xx - 3.0f * yy);
}

// dL/d(direction) of sum_k w_k Y_k(x, y, z), treating x, y, z as free polynomial variables.
__device__ __forceinline__ float3 sh_grad_dir(float x, float y, float z, int deg,
                                              const float w[16]) {
    float gx = 0.f, gy = 0.f, gz = 0.f;
    if (deg >= 1) {
        gy += SH_C1 * w[1];
        gz += SH_C1 * w[2];
        gx += SH_C1 * w[3];
    }
    if (deg >= 2) {
        gx += SH_C2A * y * w[4];              gy += SH_C2A * x * w[4];
        gy += SH_C2A * z * w[5];              gz += SH_C2A * y * w[5];
        gx += -2.f * SH_C2B * x * w[6];       gy += -2.f * SH_C2B * y * w[6];
        gz += 4.f * SH_C2B * z * w[6];
        gx += SH_C2A * z * w[7];              gz += SH_C2A * x * w[7];
        gx += 2.f * SH_C2C * x * w[8];        gy += -2.f * SH_C2C * y * w[8];
    }
    if (deg >= 3) {
        const float xx = x * x, yy = y * y, zz = z * z;
        gx += SH_C3A * 6.f * x * y * w[9];
        gy += SH_C3A * (3.f * xx - 3.f * yy) * w[9];
        gx += SH_C3B * y * z * w[10];
        gy += SH_C3B * x * z * w[10];
        gz += SH_C3B * x * y * w[10];
        gx += SH_C3C * (-2.f * x * y) * w[11];
        gy += SH_C3C * (4.f * zz - xx - 3.f * yy) * w[11];
        gz += SH_C3C * 8.f * y * z * w[11];
        gx += SH_C3D * (-6.f * x * z) * w[12];
        gy += SH_C3D * (-6.f * y * z) * w[12];
        gz += SH_C3D * (6.f * zz - 3.f * xx - 3.f * yy) * w[12];
        gx += SH_C3C * (4.f * zz - 3.f * xx - yy) * w[13];
        gy += SH_C3C * (-2.f * x * y) * w[13];
        gz += SH_C3C * 8.f * x * z * w[13];
        gx += SH_C3E * 2.f * x * z * w[14];
        gy += SH_C3E * (-2.f * y * z) * w[14];
        gz += SH_C3E * (xx - yy) * w[14];
        gx += SH_C3A * (3.f * xx - 3.f * yy) * w[15];
        gy += SH_C3A * (-6.f * x * y) * w[15];
    }
    return make_float3(gx, gy, gz);
}

// Everything the forward computes for one Gaussian, kept for the backward.
struct Geo {
    bool vis;
    float tx, ty, tz;     // camera coordinates (tz rounded from its FP64 value)
    double tzd;
    float qw, qx, qy, qz, qn;   // unit quaternion and the raw norm
    float R[9];           // rotation of the Gaussian
    float S3[6];          // Sigma_3D: xx, xy, xz, yy, yz, zz
    float T[6];           // J W (2x3, row-major)
    float sxx, sxy, syy;  // Sigma_2D with the dilation
    float det, ca, cb, cc;
    float mx, my;         // mean2d
};

__device__ __forceinline__ void geometry(const CamDev& cam, float amin, float eps2d, int W, int H,
                                         const float* __restrict__ m3, const float* __restrict__ sc,
                                         const float* __restrict__ qr, float o, Geo& g) {
    const float px = m3[0], py = m3[1], pz = m3[2];
    // View depth in FP64 (products of two floats are exact), summed left to right, rounded once:
    // the sort key therefore equals fp32 of the exact-order FP64 depth.
    g.tzd = (((double)cam.R[6] * px + (double)cam.R[7] * py) + (double)cam.R[8] * pz) +
            (double)cam.t[2];
    g.tz = (float)g.tzd;
    g.vis = (g.tzd >= (double)cam.znear) && (o >= amin);
    g.tx = cam.R[0] * px + cam.R[1] * py + cam.R[2] * pz + cam.t[0];
    g.ty = cam.R[3] * px + cam.R[4] * py + cam.R[5] * pz + cam.t[1];
    const float tz = g.vis ? g.tz : 1.0f;

    // Sigma_3D = R diag(s^2) R^T from the normalised quaternion (w, x, y, z).
    float w = qr[0], x = qr[1], y = qr[2], z = qr[3];
    g.qn = sqrtf(w * w + x * x + y * y + z * z);
    const float inv = g.qn > 0.f ? 1.0f / g.qn : 0.f;
    w *= inv; x *= inv; y *= inv; z *= inv;
    g.qw = w; g.qx = x; g.qy = y; g.qz = z;
    float* R = g.R;
    R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z);       R[2] = 2.f * (x * z + w * y);
    R[3] = 2.f * (x * y + w * z);       R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
    R[6] = 2.f * (x * z - w * y);       R[7] = 2.f * (y * z + w * x);       R[8] = 1.f - 2.f * (x * x + y * y);
    const float s0 = sc[0] * sc[0], s1 = sc[1] * sc[1], s2 = sc[2] * sc[2];
    // Sigma_3D[i][j] = sum_k R[i][k] s_k^2 R[j][k]
    g.S3[0] = R[0] * R[0] * s0 + R[1] * R[1] * s1 + R[2] * R[2] * s2;
    g.S3[1] = R[0] * R[3] * s0 + R[1] * R[4] * s1 + R[2] * R[5] * s2;
    g.S3[2] = R[0] * R[6] * s0 + R[1] * R[7] * s1 + R[2] * R[8] * s2;
    g.S3[3] = R[3] * R[3] * s0 + R[4] * R[4] * s1 + R[5] * R[5] * s2;
    g.S3[4] = R[3] * R[6] * s0 + R[4] * R[7] * s1 + R[5] * R[8] * s2;
    g.S3[5] = R[6] * R[6] * s0 + R[7] * R[7] * s1 + R[8] * R[8] * s2;

    // T = J W with J the Jacobian of (fx x/z + cx, fy y/z + cy) at t.
    const float iz = 1.0f / tz, iz2 = iz * iz;
    const float j00 = cam.fx * iz, j02 = -cam.fx * g.tx * iz2;
    const float j11 = cam.fy * iz, j12 = -cam.fy * g.ty * iz2;
    for (int j = 0; j < 3; ++j) {
        g.T[j] = j00 * cam.R[j] + j02 * cam.R[6 + j];
        g.T[3 + j] = j11 * cam.R[3 + j] + j12 * cam.R[6 + j];
    }
    const float* S = g.S3;
    const float* T = g.T;
    // U = T Sigma_3D (2x3)
    float U0[3], U1[3];
    U0[0] = T[0] * S[0] + T[1] * S[1] + T[2] * S[2];
    U0[1] = T[0] * S[1] + T[1] * S[3] + T[2] * S[4];
    U0[2] = T[0] * S[2] + T[1] * S[4] + T[2] * S[5];
    U1[0] = T[3] * S[0] + T[4] * S[1] + T[5] * S[2];
    U1[1] = T[3] * S[1] + T[4] * S[3] + T[5] * S[4];
    U1[2] = T[3] * S[2] + T[4] * S[4] + T[5] * S[5];
    g.sxx = U0[0] * T[0] + U0[1] * T[1] + U0[2] * T[2] + eps2d;
    g.sxy = U0[0] * T[3] + U0[1] * T[4] + U0[2] * T[5];
    g.syy = U1[0] * T[3] + U1[1] * T[4] + U1[2] * T[5] + eps2d;
    g.det = g.sxx * g.syy - g.sxy * g.sxy;
    const float idet = g.det > 0.f ? 1.0f / g.det : 0.f;
    g.ca = g.syy * idet;
    g.cb = -g.sxy * idet;
    g.cc = g.sxx * idet;
    g.mx = cam.fx * g.tx * iz + cam.cx;
    g.my = cam.fy * g.ty * iz + cam.cy;
    g.vis = g.vis && (g.det > 0.f);
    if (g.vis) {
        // Frustum culling: the alpha >= alpha_min ellipse's bounding box (padded against FP32
        // error) must hold a pixel centre of the image.
        const float r2 = 2.0f * logf(o / amin);
        const float hx = sqrtf(fmaxf(r2 * g.sxx, 0.f)) * 1.001f + 0.01f;
        const float hy = sqrtf(fmaxf(r2 * g.syy, 0.f)) * 1.001f + 0.01f;
        g.vis = (g.mx + hx >= 0.5f) && (g.mx - hx <= (float)W - 0.5f) &&
                (g.my + hy >= 0.5f) && (g.my - hy <= (float)H - 0.5f) &&
                isfinite(g.mx) && isfinite(g.my);
    }
}

// The NC = 3 (deg + 1)^2 SH coefficients of one Gaussian between memory and registers. With NC a
// multiple of 4 (degrees 1 and 3) every Gaussian's block starts 16-byte aligned, and one wave
// instruction moves 64 x 16 B instead of 64 x 4 B at a stride of NC floats.
template <int NC>
__device__ __forceinline__ void load_coeffs(const float* __restrict__ p, float (&c)[NC]) {
    if constexpr (NC % 4 == 0) {
        const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
        for (int j = 0; j < NC / 4; ++j) {
            const float4 v = q[j];
            c[4 * j] = v.x; c[4 * j + 1] = v.y; c[4 * j + 2] = v.z; c[4 * j + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < NC; ++j) c[j] = p[j];
    }
}

template <int NC>
__device__ __forceinline__ void store_coeffs(float* __restrict__ p, const float (&c)[NC]) {
    if constexpr (NC % 4 == 0) {
        float4* q = reinterpret_cast<float4*>(p);
#pragma unroll
        for (int j = 0; j < NC / 4; ++j) q[j] = make_float4(c[4 * j], c[4 * j + 1], c[4 * j + 2], c[4 * j + 3]);
    } else {
#pragma unroll
        for (int j = 0; j < NC; ++j) p[j] = c[j];
    }
}

template <int DEG>
__global__ __launch_bounds__(256) void k_preprocess(
    int n, const float* __restrict__ means3d, const float* __restrict__ scales,
    const float* __restrict__ quats, const float* __restrict__ opac, const float* __restrict__ sh,
    const CamSet cams, float amin, float eps2d, float* __restrict__ means2d,
    float* __restrict__ conics, float* __restrict__ rgb, float* __restrict__ depth,
    uint32_t* __restrict__ key_by_id, uint64_t vws) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const CamDev& cam = cams.c[blockIdx.y];
    means2d = view_at(means2d, 2ull * n);
    conics = view_at(conics, 3ull * n);
    rgb = view_at(rgb, 3ull * n);
    depth = view_at(depth, (uint64_t)n);
    key_by_id = view_bytes(key_by_id, vws);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        bool vis = false;
        const float o = opac[i];
        Geo g;
        geometry(cam, amin, eps2d, cam.width, cam.height, means3d + 3 * (size_t)i,
                 scales + 3 * (size_t)i, quats + 4 * (size_t)i, o, g);
        vis = g.vis;
        float c0 = 0.f, c1 = 0.f, c2 = 0.f;
        if (vis) {
            float vx = means3d[3 * (size_t)i] - cam.campos[0];
            float vy = means3d[3 * (size_t)i + 1] - cam.campos[1];
            float vz = means3d[3 * (size_t)i + 2] - cam.campos[2];
            const float il = 1.0f / sqrtf(vx * vx + vy * vy + vz * vz);
            vx *= il; vy *= il; vz *= il;
            float Y[16];
            sh_eval(vx, vy, vz, DEG, Y);
            float c[3 * K];
            load_coeffs<3 * K>(sh + (size_t)i * (3 * K), c);
            c0 = 0.5f; c1 = 0.5f; c2 = 0.5f;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                c0 += Y[k] * c[3 * k];
                c1 += Y[k] * c[3 * k + 1];
                c2 += Y[k] * c[3 * k + 2];
            }
            c0 = fmaxf(c0, 0.f); c1 = fmaxf(c1, 0.f); c2 = fmaxf(c2, 0.f);
        }
        means2d[2 * (size_t)i] = vis ? g.mx : 0.f;
        means2d[2 * (size_t)i + 1] = vis ? g.my : 0.f;
        conics[3 * (size_t)i] = vis ? g.ca : 0.f;
        conics[3 * (size_t)i + 1] = vis ? g.cb : 0.f;
        conics[3 * (size_t)i + 2] = vis ? g.cc : 0.f;
        rgb[3 * (size_t)i] = c0;
        rgb[3 * (size_t)i + 1] = c1;
        rgb[3 * (size_t)i + 2] = c2;
        depth[i] = vis ? g.tz : 0.f;
        key_by_id[i] = vis ? __float_as_uint(g.tz) : 0xFFFFFFFFu;
    }
}

template <int DEG>
__global__ __launch_bounds__(256) void k_preprocess_bwd(
    int n, const float* __restrict__ means3d, const float* __restrict__ scales,
    const float* __restrict__ quats, const float* __restrict__ opac, const float* __restrict__ sh,
    const CamSet cams, int nviews, float amin, float eps2d, const float* __restrict__ g_m2,
    const float* __restrict__ g_con, const float* __restrict__ g_rgb,
    const float* __restrict__ g_op2, float* __restrict__ d_m3, float* __restrict__ d_sc,
    float* __restrict__ d_q, float* __restrict__ d_op, float* __restrict__ d_sh) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int K = (DEG + 1) * (DEG + 1);
    const float o = opac[i];
    // sums over the views, in view order; a view that culls the splat adds nothing
    float a_m3[3] = {0.f, 0.f, 0.f}, a_sc[3] = {0.f, 0.f, 0.f}, a_q[4] = {0.f, 0.f, 0.f, 0.f};
    float a_op = 0.f;
    float a_sh[3 * K];
#pragma unroll
    for (int j = 0; j < 3 * K; ++j) a_sh[j] = 0.f;
    float co[3 * K];
    load_coeffs<3 * K>(sh + (size_t)i * (3 * K), co);
    for (int v = 0; v < nviews; ++v) {
        const CamDev& cam = cams.c[v];
        const size_t vi = (size_t)v * n + i;    // this Gaussian in view v's [n] arrays
        Geo g;
        geometry(cam, amin, eps2d, cam.width, cam.height, means3d + 3 * (size_t)i,
                 scales + 3 * (size_t)i, quats + 4 * (size_t)i, o, g);
        if (!g.vis) continue;
        // ---- conic -> Sigma_2D: G2 = -C Ghat C, Ghat = [[ga, gb/2], [gb/2, gc]] ----------------
        const float ga = g_con[3 * vi], gb = g_con[3 * vi + 1], gc = g_con[3 * vi + 2];
        const float a = g.ca, b = g.cb, c = g.cc;
        const float P00 = ga * a + 0.5f * gb * b, P01 = ga * b + 0.5f * gb * c;
        const float P10 = 0.5f * gb * a + gc * b, P11 = 0.5f * gb * b + gc * c;
        const float G00 = -(a * P00 + b * P10);
        const float G01 = -0.5f * ((a * P01 + b * P11) + (b * P00 + c * P10));
        const float G11 = -(b * P01 + c * P11);
        // ---- Sigma_2D = T S T^T: dL/dT = 2 G2 T S, dL/dS = T^T G2 T ---------------------------
        const float* T = g.T;
        const float* S = g.S3;
        float Sm[9] = {S[0], S[1], S[2], S[1], S[3], S[4], S[2], S[4], S[5]};
        float TS[6];   // T S (2x3)
        for (int r = 0; r < 2; ++r)
            for (int j = 0; j < 3; ++j)
                TS[3 * r + j] = T[3 * r] * Sm[j] + T[3 * r + 1] * Sm[3 + j] + T[3 * r + 2] * Sm[6 + j];
        float dT[6];
        for (int j = 0; j < 3; ++j) {
            dT[j] = 2.f * (G00 * TS[j] + G01 * TS[3 + j]);
            dT[3 + j] = 2.f * (G01 * TS[j] + G11 * TS[3 + j]);
        }
        float dS[9];
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l)
                dS[3 * k + l] = T[k] * (G00 * T[l] + G01 * T[3 + l]) +
                                T[3 + k] * (G01 * T[l] + G11 * T[3 + l]);
        // ---- Sigma_3D = M M^T, M = R diag(s): dL/dM = 2 dS M ----------------------------------
        const float* R = g.R;
        const float s[3] = {scales[3 * (size_t)i], scales[3 * (size_t)i + 1], scales[3 * (size_t)i + 2]};
        float dM[9];
        for (int r = 0; r < 3; ++r)
            for (int j = 0; j < 3; ++j)
                dM[3 * r + j] = 2.f * (dS[3 * r] * R[j] + dS[3 * r + 1] * R[3 + j] +
                                       dS[3 * r + 2] * R[6 + j]) * s[j];
        float dR[9];
        for (int r = 0; r < 3; ++r)
            for (int j = 0; j < 3; ++j) dR[3 * r + j] = dM[3 * r + j] * s[j];
        for (int j = 0; j < 3; ++j)
            a_sc[j] += dM[j] * R[j] + dM[3 + j] * R[3 + j] + dM[6 + j] * R[6 + j];
        // ---- R(q): derivatives of the nine entries w.r.t. the unit quaternion -------------------
        const float w = g.qw, x = g.qx, y = g.qy, z = g.qz;
        float dw = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
        float dx = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] +
                          w * dR[7] - 2.f * x * dR[8]);
        float dy = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                          z * dR[7] - 2.f * y * dR[8]);
        float dz = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] +
                          y * dR[5] + x * dR[6] + y * dR[7]);
        // through the normalisation q / |q|
        const float dot = w * dw + x * dx + y * dy + z * dz;
        const float iqn = 1.0f / g.qn;
        a_q[0] += (dw - w * dot) * iqn;
        a_q[1] += (dx - x * dot) * iqn;
        a_q[2] += (dy - y * dot) * iqn;
        a_q[3] += (dz - z * dot) * iqn;
        // ---- T = J W and mean2d: gradient w.r.t. camera coordinates -----------------------------
        const float dJ00 = dT[0] * cam.R[0] + dT[1] * cam.R[1] + dT[2] * cam.R[2];
        const float dJ02 = dT[0] * cam.R[6] + dT[1] * cam.R[7] + dT[2] * cam.R[8];
        const float dJ11 = dT[3] * cam.R[3] + dT[4] * cam.R[4] + dT[5] * cam.R[5];
        const float dJ12 = dT[3] * cam.R[6] + dT[4] * cam.R[7] + dT[5] * cam.R[8];
        const float iz = 1.0f / g.tz, iz2 = iz * iz, iz3 = iz2 * iz;
        const float gmx = g_m2[2 * vi], gmy = g_m2[2 * vi + 1];
        float dtx = dJ02 * (-cam.fx * iz2) + gmx * cam.fx * iz;
        float dty = dJ12 * (-cam.fy * iz2) + gmy * cam.fy * iz;
        float dtz = dJ00 * (-cam.fx * iz2) + dJ02 * (2.f * cam.fx * g.tx * iz3) +
                    dJ11 * (-cam.fy * iz2) + dJ12 * (2.f * cam.fy * g.ty * iz3) -
                    gmx * cam.fx * g.tx * iz2 - gmy * cam.fy * g.ty * iz2;
        float dmx = cam.R[0] * dtx + cam.R[3] * dty + cam.R[6] * dtz;
        float dmy = cam.R[1] * dtx + cam.R[4] * dty + cam.R[7] * dtz;
        float dmz = cam.R[2] * dtx + cam.R[5] * dty + cam.R[8] * dtz;
        // ---- SH colour: coefficients and the view-direction term ---------------------------------
        float vx = means3d[3 * (size_t)i] - cam.campos[0];
        float vy = means3d[3 * (size_t)i + 1] - cam.campos[1];
        float vz = means3d[3 * (size_t)i + 2] - cam.campos[2];
        const float il = 1.0f / sqrtf(vx * vx + vy * vy + vz * vz);
        const float ux = vx * il, uy = vy * il, uz = vz * il;
        float Y[16];
        sh_eval(ux, uy, uz, DEG, Y);
        float val[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
        for (int k = 0; k < K; ++k)
            for (int ch = 0; ch < 3; ++ch) val[ch] += Y[k] * co[3 * k + ch];
        float gv[3];
        for (int ch = 0; ch < 3; ++ch) gv[ch] = val[ch] > 0.f ? g_rgb[3 * vi + ch] : 0.f;
        float wY[16];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            a_sh[3 * k] += gv[0] * Y[k];
            a_sh[3 * k + 1] += gv[1] * Y[k];
            a_sh[3 * k + 2] += gv[2] * Y[k];
            wY[k] = gv[0] * co[3 * k] + gv[1] * co[3 * k + 1] + gv[2] * co[3 * k + 2];
        }
#pragma unroll
        for (int k = K; k < 16; ++k) wY[k] = 0.f;
        const float3 gd = sh_grad_dir(ux, uy, uz, DEG, wY);
        const float dd = gd.x * ux + gd.y * uy + gd.z * uz;
        dmx += (gd.x - ux * dd) * il;
        dmy += (gd.y - uy * dd) * il;
        dmz += (gd.z - uz * dd) * il;
        a_m3[0] += dmx;
        a_m3[1] += dmy;
        a_m3[2] += dmz;
        a_op += g_op2[vi];
    }
    for (int j = 0; j < 3; ++j) { d_m3[3 * (size_t)i + j] = a_m3[j]; d_sc[3 * (size_t)i + j] = a_sc[j]; }
    for (int j = 0; j < 4; ++j) d_q[4 * (size_t)i + j] = a_q[j];
    d_op[i] = a_op;
    store_coeffs<3 * K>(d_sh + (size_t)i * K * 3, a_sh);
}

// Keys for splats that arrive already projected: order-preserving uint32 of the fp32 depth;
// culled when no fragment with alpha >= alpha_min can land on a pixel centre of the image.
__global__ __launch_bounds__(256) void k_prepare_2d(
    int n, int W, int H, float amin, const float* __restrict__ means2d,
    const float* __restrict__ conics, const float* __restrict__ opac,
    const float* __restrict__ depth, uint32_t* __restrict__ key_by_id) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        bool vis = false;
        const float a = conics[3 * (size_t)i], b = conics[3 * (size_t)i + 1], c = conics[3 * (size_t)i + 2];
        const float o = opac[i];
        const float mx = means2d[2 * (size_t)i], my = means2d[2 * (size_t)i + 1];
        const float det = a * c - b * b;
        vis = a > 0.f && c > 0.f && det > 0.f && o >= amin && isfinite(mx) && isfinite(my);
        if (vis) {
            const float r2 = 2.0f * logf(o / amin);
            const float hx = sqrtf(fmaxf(r2 * c / det, 0.f)) * 1.001f + 0.01f;
            const float hy = sqrtf(fmaxf(r2 * a / det, 0.f)) * 1.001f + 0.01f;
            vis = (mx + hx >= 0.5f) && (mx - hx <= (float)W - 0.5f) && (my + hy >= 0.5f) &&
                  (my - hy <= (float)H - 0.5f);
        }
        const uint32_t u = __float_as_uint(depth[i]);
        const uint32_t k = (u & 0x80000000u) ? ~u : (u | 0x80000000u);   // monotone in the value
        key_by_id[i] = vis ? (k == 0xFFFFFFFFu ? 0xFFFFFFFEu : k) : 0xFFFFFFFFu;
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, size_t count, uint32_t value,
                           uint64_t stride) {
    p = view_bytes(p, stride);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = value;
}

hipError_t launch_fill_u32(void* p, size_t count, uint32_t value, hipStream_t s, int views,
                           uint64_t stride) {
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks, views), dim3(256), 0, s, (uint32_t*)p,
                       count, value, stride);
    return hipGetLastError();
}

CamDev make_cam(const gs_camera& c) {
    CamDev d;
    for (int r = 0; r < 3; ++r) {
        for (int j = 0; j < 3; ++j) d.R[3 * r + j] = c.viewmat[4 * r + j];
        d.t[r] = c.viewmat[4 * r + 3];
    }
    for (int j = 0; j < 3; ++j)   // campos = -R^T t, in double then rounded
        d.campos[j] = (float)(-((double)d.R[j] * d.t[0] + (double)d.R[3 + j] * d.t[1] +
                                (double)d.R[6 + j] * d.t[2]));
    d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
    d.width = c.width; d.height = c.height; d.znear = c.znear;
    return d;
}

hipError_t launch_preprocess(const CamSet& cams, const Views& vs, const gs_config& cfg, int n,
                             const float* means3d, const float* scales, const float* quats,
                             const float* opac, const float* sh, float* means2d, float* conics,
                             float* rgb, float* depth, uint32_t* keys, int32_t* ids,
                             int32_t* n_visible, void* ws, hipStream_t s) {
    if (n == 0) return launch_fill_u32(n_visible, (size_t)vs.count, 0u, s);
    uint32_t* key_by_id = (uint32_t*)ws;
    void* rest = (char*)ws + align_up((size_t)n * 4);
    decltype(&k_preprocess<3>) k = cfg.sh_degree == 0 ? k_preprocess<0>
                                  : cfg.sh_degree == 1 ? k_preprocess<1>
                                  : cfg.sh_degree == 2 ? k_preprocess<2> : k_preprocess<3>;
    hipLaunchKernelGGL(k, dim3((n + 255) / 256, vs.count), dim3(256), 0, s, n, means3d, scales,
                       quats, opac, sh, cams, cfg.alpha_min, cfg.eps2d, means2d, conics, rgb, depth,
                       key_by_id, vs.ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_compact(n, key_by_id, keys, ids, n_visible, rest, s, vs);
}

hipError_t launch_preprocess_bwd(const CamSet& cams, int nviews, const gs_config& cfg, int n,
                                 const float* means3d, const float* scales, const float* quats,
                                 const float* opac, const float* sh, const float* g_means2d,
                                 const float* g_conics, const float* g_rgb, const float* g_opac2d,
                                 float* d_means3d, float* d_scales, float* d_quats, float* d_opac,
                                 float* d_sh, hipStream_t s) {
    if (n == 0) return hipSuccess;
    decltype(&k_preprocess_bwd<3>) k = cfg.sh_degree == 0 ? k_preprocess_bwd<0>
                                      : cfg.sh_degree == 1 ? k_preprocess_bwd<1>
                                      : cfg.sh_degree == 2 ? k_preprocess_bwd<2> : k_preprocess_bwd<3>;
    hipLaunchKernelGGL(k, dim3((n + 255) / 256), dim3(256), 0, s, n, means3d, scales, quats, opac,
                       sh, cams, nviews, cfg.alpha_min, cfg.eps2d, g_means2d, g_conics, g_rgb,
                       g_opac2d, d_means3d, d_scales, d_quats, d_opac, d_sh);
    return hipGetLastError();
}

hipError_t launch_prepare_2d(int width, int height, const gs_config& cfg, int n,
                             const float* means2d, const float* conics, const float* opac,
                             const float* depth, uint32_t* keys, int32_t* ids, int32_t* n_visible,
                             void* ws, hipStream_t s) {
    if (n == 0) return launch_fill_u32(n_visible, 1, 0u, s);
    uint32_t* key_by_id = (uint32_t*)ws;
    void* rest = (char*)ws + align_up((size_t)n * 4);
    hipLaunchKernelGGL(k_prepare_2d, dim3((n + 255) / 256), dim3(256), 0, s, n, width, height,
                       cfg.alpha_min, means2d, conics, opac, depth, key_by_id);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_compact(n, key_by_id, keys, ids, n_visible, rest, s);
}

}  // namespace gsr
