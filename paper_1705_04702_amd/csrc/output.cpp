// output.cpp -- the writing phase: instrument data cubes as FITS files and
// SEDs as text files (Section 3.2, writing).  A cube file can be created
// first and filled one range of wavelength slices at a time, so that
// producers that each hold some of the wavelengths write their own slices
// into one file (the wavelength-sliced data cube of Section 5.2,
// ParallelDatacube class).
//
// FITS layout: a primary HDU with the cube, BITPIX = -64, NAXIS1 = x (fastest),
// NAXIS2 = y, NAXIS3 = wavelength, then an IMAGE extension WAVELENGTHS with
// the n_lambda wavelengths in micron.  Headers are 80-character cards in
// 2880-byte records, data big-endian IEEE doubles padded to 2880 bytes.
#include <cerrno>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mcrt.h"

namespace mcrt {
int report_error(int code, const std::string &msg); // sets mcrt_last_error()
}

namespace {

constexpr size_t kRecord = 2880;

void card(std::string &h, const char *key, const std::string &value, const char *comment = nullptr)
{
    char buf[81];
    std::string v = value;
    int n;
    if (comment)
        n = std::snprintf(buf, sizeof(buf), "%-8.8s= %20s / %s", key, v.c_str(), comment);
    else
        n = std::snprintf(buf, sizeof(buf), "%-8.8s= %20s", key, v.c_str());
    std::string c(buf, n > 80 ? 80 : (n < 0 ? 0 : n));
    c.resize(80, ' ');
    h += c;
}

std::string fits_str(const char *s)
{
    std::string v = "'";
    v += s;
    while (v.size() < 9) v += ' '; // at least 8 characters inside the quotes
    v += "'";
    // a string value starts in column 11: left-justify it in the 20-column field
    v.resize(v.size() < 20 ? 20 : v.size(), ' ');
    return v;
}

std::string fits_int(long long x) { return std::to_string(x); }

void end_header(std::string &h)
{
    std::string e = "END";
    e.resize(80, ' ');
    h += e;
    h.resize((h.size() + kRecord - 1) / kRecord * kRecord, ' ');
}

std::string primary_header(int64_t nx, int64_t ny, int64_t nl)
{
    std::string h;
    card(h, "SIMPLE", "T", "conforms to the FITS standard");
    card(h, "BITPIX", fits_int(-64), "IEEE double");
    card(h, "NAXIS", fits_int(3));
    card(h, "NAXIS1", fits_int(nx), "x pixels");
    card(h, "NAXIS2", fits_int(ny), "y pixels");
    card(h, "NAXIS3", fits_int(nl), "wavelengths (extension WAVELENGTHS)");
    card(h, "EXTEND", "T");
    card(h, "BUNIT", fits_str("flux"), "L / (4 pi d^2), source units");
    end_header(h);
    return h;
}

void put_be64(unsigned char *p, double x)
{
    uint64_t u;
    std::memcpy(&u, &x, 8);
    for (int i = 0; i < 8; ++i) p[i] = (unsigned char)(u >> (56 - 8 * i));
}

size_t padded(size_t bytes) { return (bytes + kRecord - 1) / kRecord * kRecord; }

int write_all(std::FILE *f, const void *p, size_t n) { return std::fwrite(p, 1, n, f) == n ? 0 : -1; }

int write_doubles(std::FILE *f, const double *x, size_t n)
{
    std::vector<unsigned char> buf(8 * 4096);
    size_t done = 0;
    while (done < n) {
        size_t k = n - done < 4096 ? n - done : 4096;
        for (size_t i = 0; i < k; ++i) put_be64(&buf[8 * i], x[done + i]);
        if (write_all(f, buf.data(), 8 * k)) return -1;
        done += k;
    }
    return 0;
}

int write_zeros(std::FILE *f, size_t n)
{
    std::vector<unsigned char> z(65536, 0);
    while (n) {
        size_t k = n < z.size() ? n : z.size();
        if (write_all(f, z.data(), k)) return -1;
        n -= k;
    }
    return 0;
}

} // namespace

extern "C" {

int mcrt_fits_cube_create(const char *path, int64_t nx, int64_t ny, int32_t n_lambda, const double *lambda_um)
{
    const auto fail = mcrt::report_error;
    if (!path || !lambda_um) return fail(MCRT_EINVAL, "fits_cube_create: NULL argument");
    if (nx <= 0 || ny <= 0 || n_lambda <= 0) return fail(MCRT_EINVAL, "fits_cube_create: empty cube");
    std::FILE *f = std::fopen(path, "wb");
    if (!f) return fail(MCRT_EINVAL, std::string("fits_cube_create: cannot open ") + path + ": " + std::strerror(errno));
    const std::string h = primary_header(nx, ny, n_lambda);
    const size_t data = (size_t)nx * (size_t)ny * (size_t)n_lambda * 8;
    int rc = write_all(f, h.data(), h.size());
    if (!rc) rc = write_zeros(f, padded(data));
    std::string x;
    card(x, "XTENSION", fits_str("IMAGE"), "image extension");
    card(x, "BITPIX", fits_int(-64));
    card(x, "NAXIS", fits_int(1));
    card(x, "NAXIS1", fits_int(n_lambda));
    card(x, "PCOUNT", fits_int(0));
    card(x, "GCOUNT", fits_int(1));
    card(x, "EXTNAME", fits_str("WAVELENGTHS"));
    card(x, "BUNIT", fits_str("micron"));
    end_header(x);
    if (!rc) rc = write_all(f, x.data(), x.size());
    if (!rc) rc = write_doubles(f, lambda_um, (size_t)n_lambda);
    if (!rc) rc = write_zeros(f, padded((size_t)n_lambda * 8) - (size_t)n_lambda * 8);
    if (std::fclose(f) != 0) rc = -1;
    if (rc) return fail(MCRT_EINVAL, std::string("fits_cube_create: write failed for ") + path);
    return MCRT_OK;
}

int mcrt_fits_cube_write_slices(const char *path, int64_t nx, int64_t ny, int32_t n_lambda, int32_t first,
                                int32_t count, const double *slices)
{
    const auto fail = mcrt::report_error;
    if (!path || (!slices && count > 0)) return fail(MCRT_EINVAL, "fits_cube_write_slices: NULL argument");
    if (nx <= 0 || ny <= 0 || n_lambda <= 0 || first < 0 || count < 0 || first + (int64_t)count > n_lambda)
        return fail(MCRT_EINVAL, "fits_cube_write_slices: slice range outside the cube");
    std::FILE *f = std::fopen(path, "r+b");
    if (!f) return fail(MCRT_EINVAL, std::string("fits_cube_write_slices: cannot open ") + path);
    const std::string h = primary_header(nx, ny, n_lambda);
    std::vector<char> got(h.size());
    int rc = std::fread(got.data(), 1, got.size(), f) == got.size() && std::memcmp(got.data(), h.data(), h.size()) == 0
                 ? 0
                 : -2;
    const size_t slice = (size_t)nx * (size_t)ny;
    if (!rc && std::fseek(f, (long)(h.size() + (size_t)first * slice * 8), SEEK_SET) != 0) rc = -1;
    if (!rc) rc = write_doubles(f, slices, (size_t)count * slice);
    if (std::fclose(f) != 0 && !rc) rc = -1;
    if (rc == -2) return fail(MCRT_EINVAL, "fits_cube_write_slices: the file is not a cube of this shape");
    if (rc) return fail(MCRT_EINVAL, std::string("fits_cube_write_slices: write failed for ") + path);
    return MCRT_OK;
}

int mcrt_sed_write_text(const char *path, int32_t n_lambda, const double *lambda_um, const double *sed)
{
    const auto fail = mcrt::report_error;
    if (!path || !lambda_um || !sed || n_lambda <= 0) return fail(MCRT_EINVAL, "sed_write_text: bad argument");
    std::FILE *f = std::fopen(path, "w");
    if (!f) return fail(MCRT_EINVAL, std::string("sed_write_text: cannot open ") + path);
    int rc = std::fprintf(f, "# column 1: wavelength (micron)\n# column 2: flux L / (4 pi d^2), source units\n") < 0;
    for (int32_t l = 0; l < n_lambda && !rc; ++l) rc = std::fprintf(f, "%.17g %.17g\n", lambda_um[l], sed[l]) < 0;
    if (std::fclose(f) != 0) rc = 1;
    if (rc) return fail(MCRT_EINVAL, std::string("sed_write_text: write failed for ") + path);
    return MCRT_OK;
}

} // extern "C"
